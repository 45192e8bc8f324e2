// lbm_batch.cpp -- batched drainage of many pore-throat subdomains
// (Montella et al., Sec. 2.2.2: the pore throats are solved independently).
//
// Every subdomain keeps its own buffers and node classes; one fused-step
// launch covers the live tiles of all active subdomains, and the ramp /
// bisection decisions of every subdomain are taken on the device between
// chunks of `check_every` steps.  The chunk [steps, reduction, decisions,
// state copies] is captured once as a HIP graph and replayed until no
// subdomain is running; the host only reads one counter between replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "lbm_abi.h"
#include "lbm_handle.h"
#include "sc_internal.h"

using lbmh::set_err;

namespace {

constexpr double kCs2 = 1.0 / 3.0;

struct Batch {
  int n = 0;
  hipStream_t stream = nullptr;
  std::vector<lbm_throat_t> h;
  sc::Throat *th_d = nullptr;
  sc::TileRef *tiles_d = nullptr;
  int ntiles = 0;
  int *zper_d = nullptr;  // z-periodic subdomains (ghost-plane refresh)
  int n_zper = 0;
  sc::Chunk *chunks_d = nullptr;   // reduction chunks (node-list ranges)
  int nchunks = 0;
  sc::Chunk *cchunks_d = nullptr;  // copy chunks (node ranges) of the checkpoint copies
  int ncchunks = 0;
  int *first_d = nullptr, *count_d = nullptr;
  sc::RedInfo *info_d = nullptr;
  double *partials = nullptr, *sums = nullptr, *probe = nullptr;
  sc::RampDev *rd_d = nullptr;
  sc::Ckpt *ck_d = nullptr;
  double *pc_d = nullptr, *S_d = nullptr;
  long long *steps_d = nullptr;
  int *status_d = nullptr, *nact_d = nullptr, *nact_h = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};    // autotuner trials
  hipEvent_t wall[2] = {nullptr, nullptr};  // the whole drain, first to last kernel
  std::vector<sc::Throat> th_h;
  sc::Sched sched{32, 4, 2};

  ~Batch() {
    // an error return can leave replays queued: let them finish before any
    // graph, buffer or handle they use is released
    if (stream) (void)hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void *p : {(void *)th_d, (void *)tiles_d, (void *)zper_d, (void *)chunks_d, (void *)cchunks_d,
                    (void *)first_d,
                    (void *)count_d, (void *)info_d, (void *)partials, (void *)sums,
                    (void *)probe, (void *)rd_d, (void *)ck_d, (void *)pc_d, (void *)S_d,
                    (void *)steps_d, (void *)status_d, (void *)nact_d})
      if (p) (void)hipFree(p);
    if (nact_h) (void)hipHostFree(nact_h);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto e : wall)
      if (e) (void)hipEventDestroy(e);
    for (auto x : h) lbm_throat_free(x);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

#define BCHK(call)                                                             \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      set_err("%s failed: %s", #call, hipGetErrorString(e_));                  \
      return LBM_EHIP;                                                         \
    }                                                                          \
  } while (0)

template <class T>
int dalloc(T **p, size_t count) {
  if (hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
    set_err("hipMalloc of %zu bytes failed", sizeof(T) * count);
    return LBM_ENOMEM;
  }
  return LBM_OK;
}

// tile lists of every subdomain for one launch shape
int build_tiles(Batch &B, const sc::Sched &s) {
  std::vector<sc::TileRef> tl;
  for (int t = 0; t < B.n; ++t) {
    const lbm_throat *x = B.h[t];
    sc::list_tiles(x->bricks.data(), x->n_nonsolid, x->nx, x->ny, x->nz, s.tx, s.ty, s.lz, t, tl);
    const bool tiled = s.tx != sc::kListTx;
    B.th_h[t].ntx = tiled ? (x->nx + s.tx - 1) / s.tx : 0;
    B.th_h[t].nty = tiled ? (x->ny + s.ty - 1) / s.ty : 0;
    B.th_h[t].lz = s.lz;
  }
  BCHK(hipStreamSynchronize(B.stream));
  if (B.tiles_d) (void)hipFree(B.tiles_d);
  B.tiles_d = nullptr;
  if (dalloc(&B.tiles_d, tl.size())) return LBM_ENOMEM;
  B.ntiles = (int)tl.size();
  BCHK(hipMemcpy(B.tiles_d, tl.data(), sizeof(sc::TileRef) * tl.size(), hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.th_d, B.th_h.data(), sizeof(sc::Throat) * B.n, hipMemcpyHostToDevice));
  B.sched = s;
  return LBM_OK;
}

// time candidate launch shapes over the whole batch and keep the fastest.
// Before the ramp every state is in g[0] and the checkpoint buffers are
// free: the trials advance the states with alternating buffers, as the ramp
// does, from copies in save[0] that are put back afterwards.  Each candidate
// runs an even number of steps; the close ones are timed twice.
int autotune(Batch &B, int trial_steps) {
  static const int lzs[5] = {1, 2, 4, 8, 16};
  std::vector<sc::Sched> cand;
  for (const auto &sh : sc::kShapes)
    for (int l : lzs) cand.push_back(sc::Sched{sh[0], sh[1], l});
  cand.push_back(sc::Sched{sc::kListTx, 0, 0});
  for (lbm_throat *x : B.h)
    BCHK(hipMemcpyAsync(x->save[0], x->g[0], sizeof(float) * sc::pop_elems(x->nx, x->ny, x->nz),
                        hipMemcpyDeviceToDevice, B.stream));
  std::vector<double> t(cand.size(), INFINITY);
  auto trial = [&](size_t c) -> int {
    const sc::Sched &s = cand[c];
    if (int r = build_tiles(B, s)) return r;
    int par = 0;
    auto one = [&]() {
      const hipError_t e = sc::launch_step(B.th_d, B.tiles_d, B.ntiles, s.tx, s.ty, par,
                                           B.stream, B.zper_d, B.n_zper);
      par ^= 1;
      return e;
    };
    for (int w = 0; w < 2; ++w) BCHK(one());
    BCHK(hipEventRecord(B.ev[0], B.stream));
    for (int i = 0; i < trial_steps; ++i) BCHK(one());
    BCHK(hipEventRecord(B.ev[1], B.stream));
    if (trial_steps & 1) BCHK(one());
    BCHK(hipEventSynchronize(B.ev[1]));
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, B.ev[0], B.ev[1]));
    t[c] = std::min(t[c], (double)ms);
    return LBM_OK;
  };
  // as the single-subdomain autotuner: per shape in increasing lz until a
  // segment length is 1.5x slower than the shape's best, then the candidates
  // within 1.25x of the best once more
  for (size_t c = 0; c < cand.size();) {
    double shape_best = INFINITY;
    size_t e = c;
    while (e < cand.size() && cand[e].tx == cand[c].tx && cand[e].ty == cand[c].ty) ++e;
    for (size_t k = c; k < e; ++k) {
      if (int r = trial(k)) return r;
      if (t[k] > 1.5 * shape_best) break;
      shape_best = std::min(shape_best, t[k]);
    }
    c = e;
  }
  const double first = *std::min_element(t.begin(), t.end());
  for (size_t c = 0; c < cand.size(); ++c)
    if (t[c] <= 1.25 * first)
      if (int r = trial(c)) return r;
  for (lbm_throat *x : B.h)
    BCHK(hipMemcpyAsync(x->g[0], x->save[0], sizeof(float) * sc::pop_elems(x->nx, x->ny, x->nz),
                        hipMemcpyDeviceToDevice, B.stream));
  size_t best = 0;
  for (size_t c = 1; c < cand.size(); ++c)
    if (t[c] < t[best]) best = c;
  return build_tiles(B, cand[best]);
}

// the kernels of one chunk: check_every fused steps, the reductions, the
// ramp decisions and the checkpoint copies they request
hipError_t enqueue_chunk(Batch &B, const sc::RampCfg &cfg) {
  hipError_t e = hipSuccess;
  for (int i = 0; i < cfg.every && e == hipSuccess; ++i)
    e = sc::launch_step(B.th_d, B.tiles_d, B.ntiles, B.sched.tx, B.sched.ty, i & 1, B.stream,
                        B.zper_d, B.n_zper);
  if (e == hipSuccess)
    e = sc::launch_reduce_chunks(B.th_d, B.chunks_d, B.nchunks, B.info_d, 0, B.partials, B.probe,
                                 B.stream);
  if (e == hipSuccess)
    e = sc::launch_reduce_throats(B.first_d, B.count_d, B.n, B.partials, B.sums, B.stream);
  if (e == hipSuccess)
    e = sc::launch_ramp_advance(B.th_d, B.rd_d, B.pc_d, cfg, B.sums, B.probe, B.S_d, B.steps_d,
                                B.status_d, B.n, B.nact_d, B.stream);
  if (e == hipSuccess)
    e = sc::launch_copy_requests(B.th_d, B.rd_d, B.ck_d, B.cchunks_d, B.ncchunks, 0, B.stream);
  return e;
}

int capture_chunk(Batch &B, const sc::RampCfg &cfg) {
  BCHK(hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_chunk(B, cfg);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(B.stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    set_err("graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return LBM_EHIP;
  }
  B.graph = g;
  BCHK(hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0));
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_drain_batch(int n, const lbm_params *p, const double *pc, int n_pc, const lbm_conv *c,
                    lbm_drain_result *out, lbm_batch_info *info) {
  if (n < 1 || !p || !pc || n_pc < 1 || !c || !out) {
    set_err("lbm_drain_batch: n >= 1, params, pc, conv and results are required");
    return LBM_EINVAL;
  }
  if (!(c->tol > 0) || c->check_every < 2 || (c->check_every & 1) ||
      c->max_steps < c->check_every || !(c->bisect_rel > 0)) {
    set_err("lbm_drain_batch: tol > 0, an even check_every >= 2, max_steps >= check_every and "
            "bisect_rel > 0 are required");
    return LBM_EINVAL;
  }
  for (int t = 0; t < n; ++t) {
    if (!out[t].S || !out[t].steps || !out[t].status) {
      set_err("lbm_drain_batch: result %d has no output arrays", t);
      return LBM_EINVAL;
    }
    if (p[t].probe[0] < 0) {
      set_err("lbm_drain_batch: subdomain %d has no probe node", t);
      return LBM_EINVAL;
    }
    for (int i = 0; i < n_pc; ++i) {
      const double v = pc[(size_t)t * n_pc + i];
      if (!std::isfinite(v) || !(v > 0) || (i > 0 && !(v > pc[(size_t)t * n_pc + i - 1])) ||
          !(p[t].rho_out_w + v / (kCs2 * (1.0 + p[t].G * p[t].rho_minor)) > 0)) {
        set_err("lbm_drain_batch: pc of subdomain %d must be finite, positive, strictly "
                "increasing and give a positive inlet density", t);
        return LBM_EINVAL;
      }
    }
  }
  {
    // the whole batch's device memory against the budget, before any allocation
    size_t need = 0;
    for (int t = 0; t < n; ++t) {
      if (p[t].nx < 3 || p[t].ny < 3 || p[t].nz < 3) {
        set_err("lbm_drain_batch: subdomain %d is smaller than 3 nodes on a side", t);
        return LBM_EINVAL;
      }
      need += lbmh::subdomain_bytes(p[t].nx, p[t].ny, p[t].nz, true);
    }
    if (int r = lbmh::check_budget(need, "lbm_drain_batch")) return r;
  }
  Batch B;
  B.n = n;
  BCHK(hipStreamCreate(&B.stream));
  BCHK(hipEventCreate(&B.ev[0]));
  BCHK(hipEventCreate(&B.ev[1]));
  BCHK(hipEventCreate(&B.wall[0]));
  BCHK(hipEventCreate(&B.wall[1]));
  // subdomains: geometry, initial state, checkpoints
  std::vector<sc::Chunk> chunks, cchunks;
  std::vector<int> first(n), count(n);
  std::vector<sc::RedInfo> rinfo(n);
  std::vector<sc::RampDev> rd(n);
  std::vector<sc::Ckpt> ck(n);
  B.th_h.resize(n);
  for (int t = 0; t < n; ++t) {
    lbm_params q = p[t];
    q.stream = B.stream;
    lbm_throat_t x = nullptr;
    if (int r = lbm_throat_init(&q, &x)) {
      if (r < 0) return r;
    }
    B.h.push_back(x);
    for (int i = 0; i < 2; ++i)
      if (!x->save[i] &&
          hipMalloc((void **)&x->save[i], sizeof(float) * sc::pop_elems(x->nx, x->ny, x->nz)) !=
              hipSuccess) {
        set_err("lbm_drain_batch: no device memory for the checkpoints of subdomain %d", t);
        return LBM_ENOMEM;
      }
    B.th_h[t] = x->desc;
    ck[t] = sc::Ckpt{x->save[0], x->save[1]};
    first[t] = (int)chunks.size();
    sc::list_red_chunks(t, x->nlist, chunks);
    count[t] = (int)chunks.size() - first[t];
    sc::list_chunks(t, (uint32_t)x->N, cchunks);
    rinfo[t] = sc::RedInfo{x->probe, x->phib};
    sc::RampDev R{};
    R.rho_out = x->rho_out;
    R.dpc_drho = kCs2 * (1.0 + x->G * x->rho_minor);
    R.rho_ref = x->rho_minor;
    R.n_fluid = (unsigned)x->n_fluid;
    R.phase = sc::kPhaseDone;
    rd[t] = R;
  }
  B.nchunks = (int)chunks.size();
  B.ncchunks = (int)cchunks.size();
  if (dalloc(&B.th_d, n) || dalloc(&B.chunks_d, chunks.size()) ||
      dalloc(&B.cchunks_d, cchunks.size()) || dalloc(&B.first_d, n) ||
      dalloc(&B.count_d, n) || dalloc(&B.info_d, n) || dalloc(&B.partials, 3 * chunks.size()) ||
      dalloc(&B.sums, 3 * (size_t)n) || dalloc(&B.probe, 2 * (size_t)n) || dalloc(&B.rd_d, n) ||
      dalloc(&B.ck_d, n) || dalloc(&B.pc_d, (size_t)n * n_pc) || dalloc(&B.S_d, (size_t)n * n_pc) ||
      dalloc(&B.steps_d, (size_t)n * n_pc) || dalloc(&B.status_d, (size_t)n * n_pc) ||
      dalloc(&B.nact_d, 1))
    return LBM_ENOMEM;
  if (hipHostMalloc((void **)&B.nact_h, sizeof(int), hipHostMallocDefault) != hipSuccess) {
    set_err("hipHostMalloc failed");
    return LBM_ENOMEM;
  }
  if (!cchunks.empty())
    BCHK(hipMemcpy(B.cchunks_d, cchunks.data(), sizeof(sc::Chunk) * cchunks.size(),
                   hipMemcpyHostToDevice));
  if (!chunks.empty())
    BCHK(hipMemcpy(B.chunks_d, chunks.data(), sizeof(sc::Chunk) * chunks.size(),
                 hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.first_d, first.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.count_d, count.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.info_d, rinfo.data(), sizeof(sc::RedInfo) * n, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.rd_d, rd.data(), sizeof(sc::RampDev) * n, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.ck_d, ck.data(), sizeof(sc::Ckpt) * n, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(B.pc_d, pc, sizeof(double) * n * n_pc, hipMemcpyHostToDevice));
  BCHK(hipMemset(B.S_d, 0, sizeof(double) * n * n_pc));
  BCHK(hipMemset(B.steps_d, 0, sizeof(long long) * n * n_pc));
  {
    const std::vector<int> not_run((size_t)n * n_pc, LBM_PT_NOT_RUN);
    BCHK(hipMemcpy(B.status_d, not_run.data(), sizeof(int) * n * n_pc, hipMemcpyHostToDevice));
  }
  {
    std::vector<int> zper;
    for (int t = 0; t < n; ++t)
      if (B.h[t]->per & 4) zper.push_back(t);
    if (zper.size() > 65535) {  // the ghost-plane kernel's grid y holds them
      set_err("lbm_drain_batch: at most 65535 z-periodic subdomains per batch");
      return LBM_EINVAL;
    }
    B.n_zper = (int)zper.size();
    if (dalloc(&B.zper_d, zper.size())) return LBM_ENOMEM;
    if (!zper.empty())
      BCHK(hipMemcpy(B.zper_d, zper.data(), sizeof(int) * zper.size(), hipMemcpyHostToDevice));
  }

  hipEvent_t w0 = B.wall[0], w1 = B.wall[1];
  BCHK(hipEventRecord(w0, B.stream));
  // shared launch shape, then the initial decisions
  if (int r = autotune(B, 6)) return r;
  sc::RampCfg cfg{c->tol, c->bisect_rel, c->max_steps, c->check_every, n_pc};
  BCHK(sc::launch_reduce_chunks(B.th_d, B.chunks_d, B.nchunks, B.info_d, 0, B.partials, B.probe,
                                B.stream));
  BCHK(sc::launch_reduce_throats(B.first_d, B.count_d, n, B.partials, B.sums, B.stream));
  BCHK(sc::launch_ramp_begin(B.th_d, B.rd_d, B.pc_d, cfg, B.sums, n, B.stream));
  BCHK(sc::launch_copy_requests(B.th_d, B.rd_d, B.ck_d, B.cchunks_d, B.ncchunks, 0, B.stream));
  // LBM_BATCH_NO_GRAPH=1 in the environment: the same chunk launched kernel
  // by kernel instead of replayed as a graph (for tracers that do not
  // follow graph launches); results are identical
  const char *ng = std::getenv("LBM_BATCH_NO_GRAPH");
  const bool use_graph = !(ng && ng[0] == '1');
  if (use_graph)
    if (int r = capture_chunk(B, cfg)) return r;
  // replay until every subdomain has finished its ramp; a bound on the
  // replays guards against a run that would never end
  const long long max_bisect = sc::kMaxBisect;
  const long long max_replays =
      (long long)(n_pc + max_bisect + 2) * ((c->max_steps + c->check_every - 1) / c->check_every) +
      16;
  long long replays = 0;
  const int poll = 4;
  for (;;) {
    for (int i = 0; i < poll; ++i) {
      if (use_graph)
        BCHK(hipGraphLaunch(B.exec, B.stream));
      else
        BCHK(enqueue_chunk(B, cfg));
    }
    replays += poll;
    BCHK(hipMemcpyAsync(B.nact_h, B.nact_d, sizeof(int), hipMemcpyDeviceToHost, B.stream));
    BCHK(hipStreamSynchronize(B.stream));
    if (*B.nact_h == 0) break;
    if (replays > max_replays) {
      set_err("lbm_drain_batch: ramp did not finish within %lld chunk replays", replays);
      return LBM_ESTATE;
    }
  }
  BCHK(hipEventRecord(w1, B.stream));
  BCHK(hipEventSynchronize(w1));
  float wall = 0.f;
  BCHK(hipEventElapsedTime(&wall, w0, w1));
  // results
  std::vector<double> S((size_t)n * n_pc);
  std::vector<long long> steps((size_t)n * n_pc);
  std::vector<int> status((size_t)n * n_pc);
  BCHK(hipMemcpy(rd.data(), B.rd_d, sizeof(sc::RampDev) * n, hipMemcpyDeviceToHost));
  BCHK(hipMemcpy(S.data(), B.S_d, sizeof(double) * n * n_pc, hipMemcpyDeviceToHost));
  BCHK(hipMemcpy(steps.data(), B.steps_d, sizeof(long long) * n * n_pc, hipMemcpyDeviceToHost));
  BCHK(hipMemcpy(status.data(), B.status_d, sizeof(int) * n * n_pc, hipMemcpyDeviceToHost));
  bool warn = false, failed = false;
  long long node_updates = 0, fluid_updates = 0, lattice_steps = 0;
  for (int t = 0; t < n; ++t) {
    const sc::RampDev &R = rd[t];
    for (int i = 0; i < n_pc; ++i) {
      out[t].S[i] = S[(size_t)t * n_pc + i];
      out[t].steps[i] = steps[(size_t)t * n_pc + i];
      out[t].status[i] = status[(size_t)t * n_pc + i];
    }
    out[t].invaded_at = R.invaded_at;
    out[t].n_bisect = R.n_bisect;
    out[t].total_steps = R.total_steps;
    out[t].failed = R.failed ? 1 : 0;
    if (R.failed) {  // no entry pressure from a state that became non-finite
      out[t].pce_lo = NAN;
      out[t].pce = NAN;
      out[t].pce_hi = NAN;
    } else if (R.invaded_at < 0) {
      out[t].pce_lo = pc[(size_t)t * n_pc + n_pc - 1];
      out[t].pce = NAN;
      out[t].pce_hi = INFINITY;
    } else {
      out[t].pce_lo = R.lo;
      out[t].pce_hi = R.hi;
      out[t].pce = 0.5 * (R.lo + R.hi);
    }
    warn |= R.warn != 0;
    failed |= R.failed != 0;
    node_updates += R.total_steps * (long long)B.h[t]->N;
    fluid_updates += R.total_steps * (long long)B.h[t]->n_fluid;
    lattice_steps = std::max(lattice_steps, R.total_steps);
  }
  if (info) {
    info->tx = B.sched.tx;
    info->ty = B.sched.ty;
    info->lz = B.sched.lz;
    info->replays = replays;
    info->lattice_steps = replays * c->check_every;
    info->node_updates = node_updates;
    info->fluid_updates = fluid_updates;
    info->wall_ms = wall;
    info->n_tiles = B.ntiles;
  }
  if (failed) return LBM_WPARTIAL;
  return warn ? LBM_WNOTCONV : LBM_OK;
}

}  // extern "C"
