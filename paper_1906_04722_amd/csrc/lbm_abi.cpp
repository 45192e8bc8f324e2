// lbm_abi.cpp -- host side of the C interface declared in lbm_abi.h:
// argument validation, device memory, the step/reduction launches and the
// drainage ramp with bisection (Montella et al., Sec. 2.2.2).
#include "lbm_abi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_handle.h"
#include "sc_internal.h"

namespace {
thread_local std::string g_err;
std::atomic<unsigned long long> g_budget{0};  // bytes; 0 = no budget
}  // namespace

namespace lbmh {
void set_err(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

size_t subdomain_bytes(int nx, int ny, int nz, bool checkpoints) {
  const size_t pop = sizeof(float) * sc::pop_elems(nx, ny, nz);
  const size_t N = (size_t)nx * ny * nz;
  return (checkpoints ? 4 : 2) * pop + 25 * N + ((size_t)1 << 20);
}

int check_budget(size_t need, const char *what) {
  const unsigned long long b = g_budget.load();
  if (b && need > b) {
    set_err("%s needs %zu bytes of device memory, over the budget of %llu bytes", what, need, b);
    return LBM_ENOMEM;
  }
  return LBM_OK;
}
}  // namespace lbmh

namespace {
using lbmh::set_err;

#define HIPCHK(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_err("%s failed: %s", #call, hipGetErrorString(e_));                 \
      return LBM_EHIP;                                                        \
    }                                                                         \
  } while (0)

#define TRY(call)                                                             \
  do {                                                                        \
    int r_ = (call);                                                          \
    if (r_ < 0) return r_;                                                    \
  } while (0)

constexpr double kCs2 = 1.0 / 3.0;

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

}  // namespace

namespace {

void fill_phys(lbm_throat *h) {
  sc::Phys &P = h->P;
  for (int c = 0; c < 2; ++c) {
    P.tau[c] = (float)h->tau[c];
    P.itau[c] = (float)(1.0 / h->tau[c]);
    P.Gads[c] = (float)h->Gads[c];
  }
  P.G = (float)h->G;
  // populations are stored relative to w_k rho_minor: the minority phase,
  // where populations are smallest, is then held with the most absolute
  // precision
  const double ref = h->rho_minor;
  P.rho_ref = (float)ref;
  const double rr[2][2] = {{h->rho_minor, h->rho_in}, {h->rho_out, h->rho_minor}};
  for (int i = 0; i < 2; ++i)
    for (int c = 0; c < 2; ++c) {
      P.rres[i][c] = (float)rr[i][c];
      P.gres[i][c] = (float)(rr[i][c] - ref);
    }
}

// refresh the device descriptor (buffers, sizes, tile grid, parameters)
int sync_desc(lbm_throat *h) {
  sc::Throat &T = h->desc;
  T.g[0] = h->g[0];
  T.g[1] = h->g[1];
  T.mask = h->mask;
  T.N = (uint32_t)h->N;
  T.nx = h->nx;
  T.ny = h->ny;
  T.nz = h->nz;
  T.per = h->per;
  const bool tiled = h->sched.tx != sc::kListTx;
  T.ntx = tiled ? (h->nx + h->sched.tx - 1) / h->sched.tx : 0;
  T.nty = tiled ? (h->ny + h->sched.ty - 1) / h->sched.ty : 0;
  T.lz = h->sched.lz;
  T.active = 1;
  T.list = h->list_d;
  T.nlist = h->nlist;
  T.rho = h->rho_d;
  T.P = h->P;
  HIPCHK(hipMemcpyAsync(h->desc_d, &h->desc, sizeof(sc::Throat), hipMemcpyHostToDevice,
                        h->stream));
  return LBM_OK;
}

// tiles of the current schedule that hold a non-solid node
int rebuild_tiles(lbm_throat *h) {
  std::vector<sc::TileRef> list;
  sc::list_tiles(h->bricks.data(), h->n_nonsolid, h->nx, h->ny, h->nz, h->sched.tx, h->sched.ty,
                 h->sched.lz, 0, list);
  if (list.size() > h->tiles_cap) {
    if (h->tiles_d) HIPCHK(hipStreamSynchronize(h->stream));
    if (h->tiles_d) (void)hipFree(h->tiles_d);
    h->tiles_d = nullptr;
    h->tiles_cap = 0;
    if (hipMalloc((void **)&h->tiles_d, sizeof(sc::TileRef) * std::max<size_t>(list.size(), 1)) !=
        hipSuccess) {
      set_err("hipMalloc of the tile list failed");
      return LBM_ENOMEM;
    }
    h->tiles_cap = list.size();
  }
  h->ntiles = (int)list.size();
  if (!list.empty())
    HIPCHK(hipMemcpyAsync(h->tiles_d, list.data(), sizeof(sc::TileRef) * list.size(),
                          hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return sync_desc(h);
}

int upload_rres(lbm_throat *h) {
  const double rr[4] = {h->rho_minor, h->rho_in, h->rho_out, h->rho_minor};
  HIPCHK(hipMemcpyAsync(h->rres_d, rr, sizeof rr, hipMemcpyHostToDevice, h->stream));
  return LBM_OK;
}

sc::Dom dom(const lbm_throat *h, const float *src, float *dst) {
  sc::Dom d;
  d.src = src;
  d.dst = dst;
  d.mask = h->mask;
  d.N = h->N;
  d.nx = h->nx;
  d.ny = h->ny;
  d.nz = h->nz;
  d.per = h->per;
  return d;
}

sc::Sched default_schedule(int nx, int ny, int nz) {
  sc::Sched s;
  const int w64 = (nx + 63) / 64 * 64, w32 = (nx + 31) / 32 * 32;
  s.tx = w32 < w64 ? 32 : 64;
  s.ty = s.tx == 64 ? 4 : 8;
  const long long ntx = (nx + s.tx - 1) / s.tx, nty = (ny + s.ty - 1) / s.ty;
  long long lz = (ntx * nty * nz + 1023) / 1024;
  s.lz = (int)std::max(4LL, std::min<long long>(64, lz));
  return s;
}

int validate(const lbm_params *p) {
  if (!p) {
    set_err("params is NULL");
    return LBM_EINVAL;
  }
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) {
    set_err("box %d x %d x %d: each side must be >= 3", p->nx, p->ny, p->nz);
    return LBM_EINVAL;
  }
  if ((long long)p->nx * p->ny * p->nz >= (1LL << 29)) {
    set_err("box of %lld nodes: at most 2^29 - 1 nodes per subdomain",
            (long long)p->nx * p->ny * p->nz);
    return LBM_EINVAL;
  }
  if ((long long)sc::pad_x(p->nx) * sc::pad_y(p->ny) > sc::kMaxPlaneNodes) {
    set_err("plane of %lld nodes (padded to %d x %d): at most %lld nodes per z-plane",
            (long long)p->nx * p->ny, sc::pad_x(p->nx), sc::pad_y(p->ny), sc::kMaxPlaneNodes);
    return LBM_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    const int b = p->bc[a];
    const bool ok = b == LBM_BC_PERIODIC || b == LBM_BC_WALLS || (a == 2 && b == LBM_BC_RESERVOIR);
    if (!ok) {
      set_err("bc[%d] = %d is not a boundary kind allowed on that axis", a, b);
      return LBM_EINVAL;
    }
  }
  for (int c = 0; c < 2; ++c)
    if (!(std::isfinite(p->tau[c]) && p->tau[c] > 0.5)) {
      set_err("tau[%d] = %g must be finite and > 0.5", c, p->tau[c]);
      return LBM_EINVAL;
    }
  if (!std::isfinite(p->G) || !std::isfinite(p->G_ads[0]) || !std::isfinite(p->G_ads[1])) {
    set_err("interaction strengths must be finite");
    return LBM_EINVAL;
  }
  if (!finite_pos(p->rho_major) || !finite_pos(p->rho_minor) || !finite_pos(p->rho_in_nw) ||
      !finite_pos(p->rho_out_w)) {
    set_err("densities must be finite and > 0");
    return LBM_EINVAL;
  }
  if (p->n_spheres < 0 || (p->n_spheres > 0 && !p->spheres)) {
    set_err("sphere list invalid");
    return LBM_EINVAL;
  }
  for (int i = 0; i < p->n_spheres; ++i) {
    const lbm_sphere &s = p->spheres[i];
    if (!std::isfinite(s.c[0]) || !std::isfinite(s.c[1]) || !std::isfinite(s.c[2]) ||
        !finite_pos(s.r)) {
      set_err("sphere %d has a non-finite centre or a non-positive radius", i);
      return LBM_EINVAL;
    }
  }
  if (p->prism)
    for (int a = 0; a < 3; ++a)
      if (p->prism_ids[a] < 0 || p->prism_ids[a] >= p->n_spheres) {
        set_err("prism sphere id %d out of range", p->prism_ids[a]);
        return LBM_EINVAL;
      }
  return LBM_OK;
}

void release(lbm_throat *h) {
  if (!h) return;
  for (int i = 0; i < 2; ++i) {
    if (h->g[i]) (void)hipFree(h->g[i]);
    if (h->save[i]) (void)hipFree(h->save[i]);
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    if (h->tev[i]) (void)hipEventDestroy(h->tev[i]);
  }
  if (h->mask) (void)hipFree(h->mask);
  if (h->list_d) (void)hipFree(h->list_d);
  if (h->rho_d) (void)hipFree(h->rho_d);
  if (h->types_d) (void)hipFree(h->types_d);
  if (h->rres_d) (void)hipFree(h->rres_d);
  if (h->partials) (void)hipFree(h->partials);
  if (h->chunks_d) (void)hipFree(h->chunks_d);
  if (h->redinfo_d) (void)hipFree(h->redinfo_d);
  if (h->chunk_first_d) (void)hipFree(h->chunk_first_d);
  if (h->chunk_count_d) (void)hipFree(h->chunk_count_d);
  if (h->desc_d) (void)hipFree(h->desc_d);
  if (h->tiles_d) (void)hipFree(h->tiles_d);
  if (h->zper_d) (void)hipFree(h->zper_d);
  if (h->red_d) (void)hipFree(h->red_d);
  if (h->red_h) (void)hipHostFree(h->red_h);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

int run_steps(lbm_throat *h, long long n) {
  for (long long i = 0; i < n; ++i) {
    hipError_t e = sc::launch_step(h->desc_d, h->tiles_d, h->ntiles, h->sched.tx, h->sched.ty,
                                   h->cur, h->stream, h->zper_d, h->n_zper);
    if (e != hipSuccess) {
      set_err("step launch failed: %s", hipGetErrorString(e));
      return LBM_EHIP;
    }
    h->cur = 1 - h->cur;
  }
  h->steps_done += n;
  return LBM_OK;
}

// FP64 masses, saturation and probe densities of the current state (the
// chunked reduction the batched ramp uses too, so both give the same bits)
int reduce_now(lbm_throat *h, double out[5]) {
  HIPCHK(sc::launch_reduce_chunks(h->desc_d, h->chunks_d, h->nchunks, h->redinfo_d, h->cur,
                                  h->partials, h->red_d + 3, h->stream));
  HIPCHK(sc::launch_reduce_throats(h->chunk_first_d, h->chunk_count_d, 1, h->partials, h->red_d,
                                   h->stream));
  HIPCHK(hipMemcpyAsync(h->red_h, h->red_d, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < 5; ++i) out[i] = h->red_h[i];
  out[2] = h->n_fluid ? out[2] / (double)h->n_fluid : 0.0;
  return LBM_OK;
}

int set_rho_in(lbm_throat *h, double r) {
  h->rho_in = r;
  fill_phys(h);
  TRY(sync_desc(h));
  return upload_rres(h);
}

int copy_state(lbm_throat *h, float *dst, const float *src) {
  HIPCHK(hipMemcpyAsync(dst, src, sizeof(float) * sc::pop_elems(h->nx, h->ny, h->nz),
                        hipMemcpyDeviceToDevice, h->stream));
  return LBM_OK;
}

}  // namespace

namespace lbmh {
int sync_desc(lbm_throat *h) { return ::sync_desc(h); }
int rebuild_tiles(lbm_throat *h) { return ::rebuild_tiles(h); }
int set_rho_in(lbm_throat *h, double r) { return ::set_rho_in(h, r); }
int copy_state(lbm_throat *h, float *dst, const float *src) { return ::copy_state(h, dst, src); }
}  // namespace lbmh


extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_set_memory_budget(size_t bytes) {
  g_budget.store(bytes);
  return LBM_OK;
}

int lbm_throat_init(const lbm_params *p, lbm_throat_t *out) {
  g_err.clear();
  if (!out) {
    set_err("out is NULL");
    return LBM_EINVAL;
  }
  TRY(validate(p));
  TRY(lbmh::check_budget(lbmh::subdomain_bytes(p->nx, p->ny, p->nz, false), "lbm_throat_init"));
  lbm_throat *h = new (std::nothrow) lbm_throat();
  if (!h) {
    set_err("host allocation failed");
    return LBM_ENOMEM;
  }
  h->nx = p->nx;
  h->ny = p->ny;
  h->nz = p->nz;
  h->N = (size_t)p->nx * p->ny * p->nz;
  for (int a = 0; a < 3; ++a) h->bc[a] = p->bc[a];
  h->per = (p->bc[0] == LBM_BC_PERIODIC ? 1 : 0) | (p->bc[1] == LBM_BC_PERIODIC ? 2 : 0) |
           (p->bc[2] == LBM_BC_PERIODIC ? 4 : 0);
  for (int c = 0; c < 2; ++c) {
    h->tau[c] = p->tau[c];
    h->Gads[c] = p->G_ads[c];
  }
  h->G = p->G;
  h->rho_major = p->rho_major;
  h->rho_minor = p->rho_minor;
  h->rho_in = p->rho_in_nw;
  h->rho_out = p->rho_out_w;
  h->phib = (p->rho_major - p->rho_minor) / (p->rho_major + p->rho_minor);
  fill_phys(h);
  h->sched = default_schedule(h->nx, h->ny, h->nz);

  auto fail = [&](int code) {
    release(h);
    return code;
  };
  // device memory: 2 x 152 B populations + 4 B mask + 1 B class per node
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    set_err("hipMemGetInfo failed");
    return fail(LBM_EHIP);
  }
  const size_t pop_bytes = sizeof(float) * sc::pop_elems(h->nx, h->ny, h->nz);
  const size_t need = 2 * pop_bytes + h->N * (2 * sizeof(uint32_t) + sizeof(float2) + 1) +
                      (64u << 20);
  if (need > free_b) {
    set_err("needs %zu bytes of device memory, %zu free", need, free_b);
    return fail(LBM_ENOMEM);
  }
  if (p->stream) {
    h->stream = (hipStream_t)p->stream;
  } else {
    if (hipStreamCreate(&h->stream) != hipSuccess) {
      set_err("hipStreamCreate failed");
      return fail(LBM_EHIP);
    }
    h->own_stream = true;
  }
#define ALLOC(ptr, bytes)                                                      \
  do {                                                                         \
    if (hipMalloc((void **)&(ptr), (bytes)) != hipSuccess) {                   \
      set_err("hipMalloc of %zu bytes failed", (size_t)(bytes));               \
      return fail(LBM_ENOMEM);                                                 \
    }                                                                          \
  } while (0)
  ALLOC(h->g[0], pop_bytes);
  ALLOC(h->g[1], pop_bytes);
  ALLOC(h->mask, sizeof(uint32_t) * h->N);
  ALLOC(h->types_d, h->N);
  ALLOC(h->rres_d, 4 * sizeof(double));
  if (h->per & 4) {
    const int zero = 0;
    ALLOC(h->zper_d, sizeof(int));
    if (hipMemcpy(h->zper_d, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      set_err("upload of the ghost-plane list failed");
      return fail(LBM_EHIP);
    }
    h->n_zper = 1;
  }
  ALLOC(h->redinfo_d, sizeof(sc::RedInfo));
  ALLOC(h->red_d, 5 * sizeof(double));
  ALLOC(h->desc_d, sizeof(sc::Throat));
  if (hipHostMalloc((void **)&h->red_h, 5 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    set_err("hipHostMalloc failed");
    return fail(LBM_ENOMEM);
  }
  for (int i = 0; i < 2; ++i)
    if (hipEventCreate(&h->ev[i]) != hipSuccess || hipEventCreate(&h->tev[i]) != hipSuccess) {
      set_err("hipEventCreate failed");
      return fail(LBM_EHIP);
    }

  // geometry on the device
  double *sph_d = nullptr, *rho_d = nullptr;
  const int ns = p->n_spheres;
  std::vector<double> sph(4 * (size_t)std::max(ns, 1));
  for (int i = 0; i < ns; ++i) {
    sph[4 * i + 0] = p->spheres[i].c[0];
    sph[4 * i + 1] = p->spheres[i].c[1];
    sph[4 * i + 2] = p->spheres[i].c[2];
    sph[4 * i + 3] = p->spheres[i].r;
  }
  std::vector<int> bin_start, bin_ids;
  int ncx = 0, ncy = 0, ncz = 0;
  sc::bin_spheres(sph.data(), ns, h->nx, h->ny, h->nz, bin_start, bin_ids, ncx, ncy, ncz);
  if (bin_ids.empty()) bin_ids.push_back(0);
  int *bins_d = nullptr;
  ALLOC(sph_d, sizeof(double) * sph.size());
  if (hipMalloc((void **)&bins_d, sizeof(int) * (bin_start.size() + bin_ids.size())) !=
      hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(sph_d);
    set_err("hipMalloc of the sphere bins failed");
    return fail(LBM_ENOMEM);
  }
  int rc = LBM_OK;
  do {
    if (hipMemcpyAsync(sph_d, sph.data(), sizeof(double) * sph.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(bins_d, bin_start.data(), sizeof(int) * bin_start.size(),
                       hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(bins_d + bin_start.size(), bin_ids.data(), sizeof(int) * bin_ids.size(),
                       hipMemcpyHostToDevice, h->stream) != hipSuccess) {
      rc = LBM_EHIP;
      break;
    }
    const sc::VoxBins bins{bins_d, bins_d + bin_start.size(), ncx, ncy, ncz};
    const int ids[3] = {p->prism_ids[0], p->prism_ids[1], p->prism_ids[2]};
    const int safe_ids[3] = {p->prism ? ids[0] : 0, p->prism ? ids[1] : 0, p->prism ? ids[2] : 0};
    if (sc::launch_voxelize(sph_d, bins, p->prism ? 1 : 0, safe_ids, h->nx, h->ny, h->nz,
                            p->bc[2] == LBM_BC_RESERVOIR, h->types_d, h->stream) != hipSuccess ||
        sc::launch_links(h->types_d, h->nx, h->ny, h->nz, h->per, h->mask, h->stream) !=
            hipSuccess) {
      rc = LBM_EHIP;
      break;
    }
    h->types.resize(h->N);
    if (hipMemcpyAsync(h->types.data(), h->types_d, h->N, hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      rc = LBM_EHIP;
      break;
    }
  } while (0);
  if (rc == LBM_OK && hipStreamSynchronize(h->stream) != hipSuccess) rc = LBM_EHIP;
  (void)hipFree(sph_d);
  (void)hipFree(bins_d);
  if (rc != LBM_OK) {
    set_err("geometry setup failed");
    return fail(rc);
  }
  long long nf = 0;
  for (size_t n = 0; n < h->N; ++n) nf += h->types[n] == sc::kFluid;
  h->n_fluid = nf;
  sc::brick_map(h->types.data(), h->nx, h->ny, h->nz, h->bricks, h->n_nonsolid);

  if (p->probe[0] >= 0) {
    if (p->probe[0] >= h->nx || p->probe[1] < 0 || p->probe[1] >= h->ny || p->probe[2] < 0 ||
        p->probe[2] >= h->nz) {
      set_err("probe node outside the box");
      return fail(LBM_EINVAL);
    }
    h->probe = (long long)p->probe[0] +
               (long long)h->nx * ((long long)p->probe[1] + (long long)h->ny * p->probe[2]);
    if (h->types[h->probe] != sc::kFluid) {
      set_err("probe node is not a fluid node");
      return fail(LBM_EINVAL);
    }
  }
  {
    const sc::RedInfo ri{h->probe, h->phib};
    if (hipMemcpy(h->redinfo_d, &ri, sizeof ri, hipMemcpyHostToDevice) != hipSuccess) {
      set_err("upload of the reduction info failed");
      return fail(LBM_EHIP);
    }
  }
  if (p->rho_init) {
    for (int c = 0; c < 2; ++c)
      for (size_t n = 0; n < h->N; ++n)
        if (h->types[n] == sc::kFluid && !finite_pos(p->rho_init[c * h->N + n])) {
          set_err("rho_init is not finite and positive on fluid node %zu", n);
          return fail(LBM_EINVAL);
        }
    ALLOC(rho_d, sizeof(double) * 2 * h->N);
    if (hipMemcpyAsync(rho_d, p->rho_init, sizeof(double) * 2 * h->N, hipMemcpyHostToDevice,
                       h->stream) != hipSuccess) {
      (void)hipFree(rho_d);
      set_err("rho_init upload failed");
      return fail(LBM_EHIP);
    }
  }
  if (upload_rres(h) != LBM_OK) {
    if (rho_d) (void)hipFree(rho_d);
    return fail(LBM_EHIP);
  }
  const sc::Dom d = dom(h, nullptr, nullptr);
  hipError_t e = sc::launch_init(d, h->P, rho_d, h->rho_major, h->rho_minor, p->z_front, h->rres_d,
                                 h->g[0], h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->g[1], 0, pop_bytes, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (rho_d) (void)hipFree(rho_d);
  if (e != hipSuccess) {
    set_err("initial state failed: %s", hipGetErrorString(e));
    return fail(LBM_EHIP);
  }
  // node list of the non-solid nodes and the density array of the node-list
  // path (solid entries stay zero: they are the stencil's solid density)
  {
    std::vector<uint32_t> list;
    list.reserve(h->n_nonsolid);
    // in storage order (brick by brick), so that the lanes of a wavefront
    // read and write whole lines of the population buffers
    const size_t nxy = (size_t)h->nx * h->ny;
    for (int z = 0; z < h->nz; ++z)
      for (int by = -sc::kOY; by < h->ny; by += sc::kBY)
        for (int bx = -sc::kOX; bx < h->nx; bx += sc::kBX)
          for (int y = std::max(by, 0); y < std::min(by + sc::kBY, h->ny); ++y)
            for (int x = std::max(bx, 0); x < std::min(bx + sc::kBX, h->nx); ++x) {
              const size_t n = (size_t)z * nxy + (size_t)y * h->nx + x;
              if (h->types[n] != sc::kSolid) list.push_back((uint32_t)n);
            }
    h->nlist = (uint32_t)list.size();
    // each entry carries the node's mask word, which saves the list kernels
    // one dependent load
    ALLOC(h->list_d, sizeof(uint2) * std::max<size_t>(list.size(), 1));
    ALLOC(h->rho_d, sizeof(float2) * h->N);
    uint32_t *ids_d = nullptr;
    ALLOC(ids_d, sizeof(uint32_t) * std::max<size_t>(list.size(), 1));
    const bool ok =
        (list.empty() ||
         (hipMemcpyAsync(ids_d, list.data(), sizeof(uint32_t) * list.size(),
                         hipMemcpyHostToDevice, h->stream) == hipSuccess &&
          sc::launch_list_entries(ids_d, h->mask, h->nlist, h->list_d, h->stream) ==
              hipSuccess)) &&
        hipMemsetAsync(h->rho_d, 0, sizeof(float2) * h->N, h->stream) == hipSuccess &&
        hipStreamSynchronize(h->stream) == hipSuccess;
    (void)hipFree(ids_d);
    if (!ok) {
      set_err("node list upload failed");
      return fail(LBM_EHIP);
    }
  }
  // reduction chunks over the node list
  {
    std::vector<sc::Chunk> ch;
    sc::list_red_chunks(0, h->nlist, ch);
    h->nchunks = (int)ch.size();
    ALLOC(h->chunks_d, sizeof(sc::Chunk) * std::max<size_t>(ch.size(), 1));
    ALLOC(h->partials, sizeof(double) * 3 * std::max<size_t>(ch.size(), 1));
    ALLOC(h->chunk_first_d, sizeof(int));
    ALLOC(h->chunk_count_d, sizeof(int));
    const int first = 0, cnt = h->nchunks;
    if ((!ch.empty() && hipMemcpy(h->chunks_d, ch.data(), sizeof(sc::Chunk) * ch.size(),
                                  hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(h->chunk_first_d, &first, sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->chunk_count_d, &cnt, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      set_err("upload of the reduction chunks failed");
      return fail(LBM_EHIP);
    }
  }
  h->cur = 0;
  if (rebuild_tiles(h) != LBM_OK) return fail(LBM_EHIP);
  *out = h;
  return LBM_OK;
#undef ALLOC
}

void lbm_throat_free(lbm_throat_t h) { release(h); }

int lbm_step(lbm_throat_t h, long long nsteps) {
  if (!h || nsteps < 0) {
    set_err("lbm_step: bad handle or negative step count");
    return LBM_EINVAL;
  }
  return run_steps(h, nsteps);
}

int lbm_sync(lbm_throat_t h) {
  if (!h) {
    set_err("NULL handle");
    return LBM_EINVAL;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_set_rho_in(lbm_throat_t h, double r) {
  if (!h || !finite_pos(r)) {
    set_err("lbm_set_rho_in: bad handle or density");
    return LBM_EINVAL;
  }
  return set_rho_in(h, r);
}

double lbm_rho_in_for_pc(lbm_throat_t h, double pc) {
  if (!h) return NAN;
  return h->rho_out + pc / (kCs2 * (1.0 + h->G * h->rho_minor));
}

long long lbm_nodes(lbm_throat_t h) { return h ? (long long)h->N : -1; }

int lbm_get_types(lbm_throat_t h, unsigned char *types) {
  if (!h || !types) {
    set_err("lbm_get_types: NULL argument");
    return LBM_EINVAL;
  }
  std::memcpy(types, h->types.data(), h->N);
  return LBM_OK;
}

int lbm_get_populations(lbm_throat_t h, double *f) {
  if (!h || !f) {
    set_err("lbm_get_populations: NULL argument");
    return LBM_EINVAL;
  }
  double *fd = nullptr;
  if (hipMalloc((void **)&fd, sizeof(double) * 38 * h->N) != hipSuccess) {
    set_err("hipMalloc for the export failed");
    return LBM_ENOMEM;
  }
  const sc::Dom d = dom(h, h->g[h->cur], nullptr);
  hipError_t e = sc::launch_export(d, h->P, h->rres_d, fd, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(f, fd, sizeof(double) * 38 * h->N, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(fd);
  if (e != hipSuccess) {
    set_err("export failed: %s", hipGetErrorString(e));
    return LBM_EHIP;
  }
  return LBM_OK;
}

int lbm_get_density(lbm_throat_t h, double *rho) {
  if (!h || !rho) {
    set_err("lbm_get_density: NULL argument");
    return LBM_EINVAL;
  }
  double *rd = nullptr;
  if (hipMalloc((void **)&rd, sizeof(double) * 2 * h->N) != hipSuccess) {
    set_err("hipMalloc for the density read-back failed");
    return LBM_ENOMEM;
  }
  const sc::Dom d = dom(h, h->g[h->cur], nullptr);
  hipError_t e = sc::launch_density(d, h->P, h->rres_d, rd, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rho, rd, sizeof(double) * 2 * h->N, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(rd);
  if (e != hipSuccess) {
    set_err("density read-back failed: %s", hipGetErrorString(e));
    return LBM_EHIP;
  }
  return LBM_OK;
}

int lbm_get_density_noalloc(lbm_throat_t h, double *rho) {
  if (!h || !rho) {
    set_err("lbm_get_density_noalloc: NULL argument");
    return LBM_EINVAL;
  }
  if (h->N > sc::kScratchNodes) {
    set_err("lbm_get_density_noalloc: %zu nodes exceed the fixed staging array of %zu nodes",
            h->N, sc::kScratchNodes);
    return LBM_EINVAL;
  }
  double *stage = nullptr;
  hipError_t e = sc::scratch_address(&stage);
  if (e != hipSuccess) {
    set_err("lbm_get_density_noalloc: no address for the staging array: %s",
            hipGetErrorString(e));
    return LBM_EHIP;
  }
  // k_density writes all 2 N values, so nothing left by an earlier call is read
  const sc::Dom d = dom(h, h->g[h->cur], nullptr);
  e = sc::launch_density(d, h->P, h->rres_d, stage, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rho, stage, sizeof(double) * 2 * h->N, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    set_err("lbm_get_density_noalloc: read-back failed: %s", hipGetErrorString(e));
    return LBM_EHIP;
  }
  return LBM_OK;
}

int lbm_reduce(lbm_throat_t h, double *mass2, double *S_w) {
  if (!h) {
    set_err("NULL handle");
    return LBM_EINVAL;
  }
  double r[5];
  TRY(reduce_now(h, r));
  if (mass2) {
    mass2[0] = r[0];
    mass2[1] = r[1];
  }
  if (S_w) *S_w = r[2];
  return LBM_OK;
}

int lbm_probe_invaded(lbm_throat_t h, int *invaded) {
  if (!h || !invaded) {
    set_err("NULL argument");
    return LBM_EINVAL;
  }
  if (h->probe < 0) {
    set_err("the handle has no probe node");
    return LBM_ESTATE;
  }
  double r[5];
  TRY(reduce_now(h, r));
  *invaded = r[4] > r[3] ? 1 : 0;
  return LBM_OK;
}

}  // extern "C"

namespace {

// ---- the drainage ramp of one subdomain as a resumable state machine -----
// Sec. 2.2.2: the capillary pressures are visited in increasing order, each
// held until the wetting saturation settles; the first invaded interval is
// bisected from the last stable state.  The machine advances in chunks of
// check_every steps, so a caller can stop it after any chunk, save the
// handle (lbm_save) and resume it in another handle (lbm_load); run to the
// end in one call it is lbm_drain_throat.

int check_drain_args(lbm_throat *h, const double *pc, int n_pc, const lbm_conv *c,
                     const char *who) {
  if (!h || !pc || n_pc < 1 || !c) {
    set_err("%s: NULL argument or n_pc < 1", who);
    return LBM_EINVAL;
  }
  if (!(c->tol > 0) || c->check_every < 1 || c->max_steps < c->check_every ||
      !(c->bisect_rel > 0)) {
    set_err("%s: invalid convergence settings", who);
    return LBM_EINVAL;
  }
  if (h->probe < 0) {
    set_err("%s needs a probe node", who);
    return LBM_ESTATE;
  }
  for (int i = 0; i < n_pc; ++i) {
    if (!std::isfinite(pc[i]) || !(pc[i] > 0) || !(lbm_rho_in_for_pc(h, pc[i]) > 0) ||
        (i > 0 && !(pc[i] > pc[i - 1]))) {
      set_err("%s: pc must be finite, positive, strictly increasing and give a positive inlet "
              "density", who);
      return LBM_EINVAL;
    }
  }
  return LBM_OK;
}

int ensure_checkpoints(lbm_throat *h, const char *who) {
  if (!h->save[0] || !h->save[1])
    TRY(lbmh::check_budget(lbmh::subdomain_bytes(h->nx, h->ny, h->nz, true), who));
  for (int i = 0; i < 2; ++i)
    if (!h->save[i] &&
        hipMalloc((void **)&h->save[i], sizeof(float) * sc::pop_elems(h->nx, h->ny, h->nz)) !=
            hipSuccess) {
      set_err("hipMalloc of a ramp checkpoint failed");
      return LBM_ENOMEM;
    }
  return LBM_OK;
}

// a run to steady state starts: the saturation it is compared against
int run_start(lbm_throat *h) {
  double r[5];
  TRY(reduce_now(h, r));
  h->ramp.S_old = r[2];
  h->ramp.run_steps = 0;
  return LBM_OK;
}

// one chunk of check_every steps of the run in progress; *ended = 1 when the
// run has ended, with its status, saturation and invasion test
int run_chunk(lbm_throat *h, int *ended, int *st, double *S, int *inv) {
  HostRamp &R = h->ramp;
  double r[5];
  if (h->timing) HIPCHK(hipEventRecord(h->tev[0], h->stream));
  TRY(run_steps(h, R.c.check_every));
  if (h->timing) HIPCHK(hipEventRecord(h->tev[1], h->stream));
  R.run_steps += R.c.check_every;
  TRY(reduce_now(h, r));
  if (h->timing) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->tev[0], h->tev[1]));
    h->timed_ms += ms;
    h->timed_launches += R.c.check_every;
  }
  const double S_new = r[2];
  *ended = 1;
  if (!std::isfinite(S_new))
    *st = LBM_PT_NONFINITE;
  else if (std::fabs(S_new - R.S_old) < R.c.tol)
    *st = LBM_PT_CONVERGED;
  else if (R.run_steps >= R.c.max_steps)
    *st = LBM_PT_NOT_CONVERGED;
  else
    *ended = 0;
  *S = S_new;
  *inv = r[4] > r[3] ? 1 : 0;
  if (!*ended) R.S_old = S_new;
  return LBM_OK;
}

int ramp_next_point(lbm_throat *h) {
  HostRamp &R = h->ramp;
  R.point += 1;
  if (R.point >= (int)R.pc.size()) {
    R.phase = HostRamp::kDone;
    return LBM_OK;
  }
  R.phase = HostRamp::kRamp;
  TRY(set_rho_in(h, lbm_rho_in_for_pc(h, R.pc[R.point])));
  return run_start(h);
}

// the next bisection run from the last stable state, or the end of the
// bisection: back to the invaded ramp state and on to the next point
int ramp_bisect_or_resume(lbm_throat *h) {
  HostRamp &R = h->ramp;
  if ((R.hi - R.lo) / R.hi > R.c.bisect_rel) {
    if (R.runs < sc::kMaxBisect) {
      ++R.runs;
      R.mid = 0.5 * (R.lo + R.hi);
      R.phase = HostRamp::kBisect;
      TRY(copy_state(h, h->g[h->cur], h->save[0]));
      TRY(set_rho_in(h, lbm_rho_in_for_pc(h, R.mid)));
      return run_start(h);
    }
    R.warn = 1;  // bracket left wider than asked (a throat invaded at pc[0])
  }
  TRY(copy_state(h, h->g[h->cur], h->save[1]));
  TRY(set_rho_in(h, R.main_rho_in));
  return ramp_next_point(h);
}

int ramp_begin(lbm_throat *h, const double *pc, int n_pc, const lbm_conv *c) {
  TRY(ensure_checkpoints(h, "lbm_drain"));
  HostRamp R;
  R.pc.assign(pc, pc + n_pc);
  R.c = *c;
  R.S.assign(n_pc, 0.0);
  R.steps.assign(n_pc, 0);
  R.status.assign(n_pc, LBM_PT_NOT_RUN);
  R.phase = HostRamp::kRamp;
  R.point = 0;
  h->ramp = std::move(R);
  TRY(copy_state(h, h->save[0], h->g[h->cur]));
  TRY(set_rho_in(h, lbm_rho_in_for_pc(h, h->ramp.pc[0])));
  return run_start(h);
}

// advance by whole chunks until the ramp is done or max_steps lattice steps
// have run in this call
int ramp_advance(lbm_throat *h, long long max_steps) {
  HostRamp &R = h->ramp;
  long long ran = 0;
  while (R.phase == HostRamp::kRamp || R.phase == HostRamp::kBisect) {
    if (ran >= max_steps) break;
    int ended = 0, st = 0, inv = 0;
    double S = 0.0;
    TRY(run_chunk(h, &ended, &st, &S, &inv));
    ran += R.c.check_every;
    if (!ended) continue;
    if (st == LBM_PT_NONFINITE) {
      set_err("the state became non-finite %s", R.phase == HostRamp::kBisect
                                                    ? "while bisecting"
                                                    : "at a ramp point");
      R.failed = 1;
      R.phase = HostRamp::kDone;
      if (R.point < (int)R.status.size() && R.status[R.point] == LBM_PT_NOT_RUN)
        R.status[R.point] = LBM_PT_NONFINITE;
      for (size_t j = R.point + 1; j < R.status.size(); ++j) R.status[j] = LBM_PT_NONFINITE;
      return LBM_ENONFINITE;
    }
    if (R.phase == HostRamp::kRamp) {
      const int i = R.point;
      R.S[i] = S;
      R.steps[i] = R.run_steps;
      R.status[i] = st;
      R.total += R.run_steps;
      R.warn |= st == LBM_PT_NOT_CONVERGED;
      if (!inv) {
        TRY(copy_state(h, h->save[0], h->g[h->cur]));
        R.stable_pc = R.pc[i];
        TRY(ramp_next_point(h));
      } else if (R.inv_at >= 0) {
        TRY(ramp_next_point(h));
      } else {
        R.inv_at = i;
        R.lo = i == 0 ? 0.0 : R.stable_pc;
        R.hi = R.pc[i];
        R.main_rho_in = h->rho_in;
        R.runs = 0;
        TRY(copy_state(h, h->save[1], h->g[h->cur]));
        TRY(ramp_bisect_or_resume(h));
      }
    } else {  // a bisection run ended
      R.total += R.run_steps;
      ++R.n_bisect;
      if (inv) {
        R.hi = R.mid;
      } else {
        R.lo = R.mid;
        TRY(copy_state(h, h->save[0], h->g[h->cur]));
      }
      TRY(ramp_bisect_or_resume(h));
    }
  }
  return LBM_OK;
}

void ramp_result(const lbm_throat *h, lbm_drain_result *out) {
  const HostRamp &R = h->ramp;
  const int n = (int)R.pc.size();
  for (int i = 0; i < n; ++i) {
    out->S[i] = R.S[i];
    out->steps[i] = R.steps[i];
    out->status[i] = R.status[i];
  }
  out->invaded_at = R.inv_at;
  out->n_bisect = R.n_bisect;
  out->total_steps = R.total;
  out->failed = R.failed;
  if (R.failed) {
    out->pce_lo = out->pce = out->pce_hi = NAN;
  } else if (R.inv_at < 0) {
    out->pce_lo = n ? R.pc[n - 1] : NAN;
    out->pce = NAN;
    out->pce_hi = INFINITY;
  } else {
    out->pce_lo = R.lo;
    out->pce_hi = R.hi;
    out->pce = 0.5 * (R.lo + R.hi);
  }
}

}  // namespace

extern "C" {

int lbm_drain_throat(lbm_throat_t h, const double *pc, int n_pc, const lbm_conv *c,
                     lbm_drain_result *out) {
  if (!out || !out->S || !out->steps || !out->status) {
    set_err("lbm_drain_throat: NULL result arrays");
    return LBM_EINVAL;
  }
  TRY(check_drain_args(h, pc, n_pc, c, "lbm_drain_throat"));
  TRY(ramp_begin(h, pc, n_pc, c));
  TRY(ramp_advance(h, LLONG_MAX));
  HIPCHK(hipStreamSynchronize(h->stream));
  ramp_result(h, out);
  return h->ramp.warn ? LBM_WNOTCONV : LBM_OK;
}

int lbm_drain_begin(lbm_throat_t h, const double *pc, int n_pc, const lbm_conv *c) {
  TRY(check_drain_args(h, pc, n_pc, c, "lbm_drain_begin"));
  return ramp_begin(h, pc, n_pc, c);
}

int lbm_drain_advance(lbm_throat_t h, long long max_steps, int *done) {
  if (!h || max_steps < 0) {
    set_err("lbm_drain_advance: NULL handle or negative step budget");
    return LBM_EINVAL;
  }
  if (h->ramp.phase == HostRamp::kIdle) {
    set_err("lbm_drain_advance: no drainage ramp begun on this handle");
    return LBM_ESTATE;
  }
  TRY(ramp_advance(h, max_steps));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (done) *done = h->ramp.phase == HostRamp::kDone ? 1 : 0;
  return LBM_OK;
}

int lbm_drain_get(lbm_throat_t h, int n_pc, lbm_drain_result *out, int *done) {
  if (!h || !out || !out->S || !out->steps || !out->status) {
    set_err("lbm_drain_get: NULL argument");
    return LBM_EINVAL;
  }
  if (h->ramp.phase == HostRamp::kIdle) {
    set_err("lbm_drain_get: no drainage ramp begun on this handle");
    return LBM_ESTATE;
  }
  if (n_pc != (int)h->ramp.pc.size()) {
    set_err("lbm_drain_get: the ramp has %d points, not %d", (int)h->ramp.pc.size(), n_pc);
    return LBM_EINVAL;
  }
  ramp_result(h, out);
  if (done) *done = h->ramp.phase == HostRamp::kDone ? 1 : 0;
  return h->ramp.warn ? LBM_WNOTCONV : LBM_OK;
}

}  // extern "C"

namespace {

// ---- checkpoint files (lbm_save / lbm_load) --------------------------------
constexpr char kMagic[8] = {'L', 'B', 'M', 'S', 'C', 'v', '1', '\0'};
constexpr size_t kIoChunk = (size_t)16 << 20;  // floats per host staging chunk

uint64_t types_hash(const std::vector<uint8_t> &t) {
  uint64_t x = 1469598103934665603ULL;  // FNV-1a, 64 bit
  for (uint8_t b : t) {
    x ^= b;
    x *= 1099511628211ULL;
  }
  return x;
}

struct File {
  FILE *f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
  template <class T>
  bool put(const T &v) { return fwrite(&v, sizeof(T), 1, f) == 1; }
  template <class T>
  bool put_n(const T *v, size_t n) { return n == 0 || fwrite(v, sizeof(T), n, f) == n; }
  template <class T>
  bool get(T &v) { return fread(&v, sizeof(T), 1, f) == 1; }
  template <class T>
  bool get_n(T *v, size_t n) { return n == 0 || fread(v, sizeof(T), n, f) == n; }
};

// the fixed part of a subdomain that a saved state must match
struct Header {
  char magic[8];
  int32_t nx, ny, nz, per;
  uint64_t N, pop_elems, types;
  double tau[2], G, Gads[2], rho_major, rho_minor, rho_out;
};

Header header_of(const lbm_throat *h) {
  Header H;
  std::memset(&H, 0, sizeof H);
  std::memcpy(H.magic, kMagic, sizeof kMagic);
  H.nx = h->nx;
  H.ny = h->ny;
  H.nz = h->nz;
  H.per = h->per;
  H.N = h->N;
  H.pop_elems = sc::pop_elems(h->nx, h->ny, h->nz);
  H.types = types_hash(h->types);
  H.tau[0] = h->tau[0];
  H.tau[1] = h->tau[1];
  H.G = h->G;
  H.Gads[0] = h->Gads[0];
  H.Gads[1] = h->Gads[1];
  H.rho_major = h->rho_major;
  H.rho_minor = h->rho_minor;
  H.rho_out = h->rho_out;
  return H;
}

bool put_ramp(File &F, const HostRamp &R) {
  const int32_t n = (int32_t)R.pc.size();
  bool ok = F.put((int32_t)R.phase) && F.put((int32_t)R.point) && F.put(n) && F.put(R.c.tol) &&
            F.put((int32_t)R.c.check_every) && F.put((int64_t)R.c.max_steps) &&
            F.put(R.c.bisect_rel) && F.put((int64_t)R.run_steps) && F.put(R.S_old) &&
            F.put(R.stable_pc) && F.put(R.lo) && F.put(R.hi) && F.put(R.mid) &&
            F.put(R.main_rho_in) && F.put((int32_t)R.inv_at) && F.put((int32_t)R.n_bisect) &&
            F.put((int32_t)R.runs) && F.put((int32_t)R.warn) && F.put((int32_t)R.failed) &&
            F.put((int64_t)R.total);
  ok = ok && F.put_n(R.pc.data(), n) && F.put_n(R.S.data(), n);
  for (int i = 0; ok && i < n; ++i) ok = F.put((int64_t)R.steps[i]) && F.put((int32_t)R.status[i]);
  return ok;
}

bool get_ramp(File &F, HostRamp &R) {
  int32_t phase, point, n, every, inv_at, n_bis, runs, warn, failed;
  int64_t max_steps, run_steps, total;
  bool ok = F.get(phase) && F.get(point) && F.get(n) && F.get(R.c.tol) && F.get(every) &&
            F.get(max_steps) && F.get(R.c.bisect_rel) && F.get(run_steps) && F.get(R.S_old) &&
            F.get(R.stable_pc) && F.get(R.lo) && F.get(R.hi) && F.get(R.mid) &&
            F.get(R.main_rho_in) && F.get(inv_at) && F.get(n_bis) && F.get(runs) && F.get(warn) &&
            F.get(failed) && F.get(total);
  if (!ok || n < 0 || n > (1 << 24) || phase < HostRamp::kIdle || phase > HostRamp::kDone)
    return false;
  R.phase = phase;
  R.point = point;
  R.c.check_every = every;
  R.c.max_steps = max_steps;
  R.run_steps = run_steps;
  R.inv_at = inv_at;
  R.n_bisect = n_bis;
  R.runs = runs;
  R.warn = warn;
  R.failed = failed;
  R.total = total;
  R.pc.resize(n);
  R.S.resize(n);
  R.steps.resize(n);
  R.status.resize(n);
  ok = F.get_n(R.pc.data(), n) && F.get_n(R.S.data(), n);
  for (int i = 0; ok && i < n; ++i) {
    int64_t st64 = 0;
    int32_t st32 = 0;
    ok = F.get(st64) && F.get(st32);
    R.steps[i] = st64;
    R.status[i] = st32;
  }
  return ok && (R.phase == HostRamp::kIdle || (n >= 1 && point >= 0 && point <= n));
}

// one device buffer of pop_elems floats to or from the file, in chunks
int buffer_out(lbm_throat *h, File &F, const float *dev, size_t n) {
  std::vector<float> tmp(std::min(n, kIoChunk));
  for (size_t o = 0; o < n; o += kIoChunk) {
    const size_t k = std::min(kIoChunk, n - o);
    HIPCHK(hipMemcpyAsync(tmp.data(), dev + o, sizeof(float) * k, hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (!F.put_n(tmp.data(), k)) {
      set_err("lbm_save: write failed");
      return LBM_EIO;
    }
  }
  return LBM_OK;
}

int buffer_in(lbm_throat *h, File &F, float *dev, size_t n) {
  std::vector<float> tmp(std::min(n, kIoChunk));
  for (size_t o = 0; o < n; o += kIoChunk) {
    const size_t k = std::min(kIoChunk, n - o);
    if (!F.get_n(tmp.data(), k)) {
      set_err("lbm_load: the file ends inside a population buffer");
      return LBM_EIO;
    }
    HIPCHK(hipMemcpyAsync(dev + o, tmp.data(), sizeof(float) * k, hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_save(lbm_throat_t h, const char *path) {
  if (!h || !path) {
    set_err("lbm_save: NULL argument");
    return LBM_EINVAL;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  File F;
  F.f = fopen(path, "wb");
  if (!F.f) {
    set_err("lbm_save: cannot open %s for writing", path);
    return LBM_EIO;
  }
  const Header H = header_of(h);
  const bool with_ckpt = h->ramp.phase == HostRamp::kRamp || h->ramp.phase == HostRamp::kBisect;
  const int32_t nbuf = with_ckpt ? 3 : 1;
  if (!F.put(H) || !F.put(h->rho_in) || !F.put((int64_t)h->steps_done) || !put_ramp(F, h->ramp) ||
      !F.put(nbuf)) {
    set_err("lbm_save: write to %s failed", path);
    return LBM_EIO;
  }
  const size_t n = sc::pop_elems(h->nx, h->ny, h->nz);
  TRY(buffer_out(h, F, h->g[h->cur], n));
  if (with_ckpt) {
    TRY(buffer_out(h, F, h->save[0], n));
    TRY(buffer_out(h, F, h->save[1], n));
  }
  if (fflush(F.f) != 0) {
    set_err("lbm_save: write to %s failed", path);
    return LBM_EIO;
  }
  return LBM_OK;
}

int lbm_load(lbm_throat_t h, const char *path) {
  if (!h || !path) {
    set_err("lbm_load: NULL argument");
    return LBM_EINVAL;
  }
  File F;
  F.f = fopen(path, "rb");
  if (!F.f) {
    set_err("lbm_load: cannot open %s", path);
    return LBM_EIO;
  }
  Header H{};
  double rho_in = 0.0;
  int64_t steps_done = 0;
  HostRamp R;
  int32_t nbuf = 0;
  if (!F.get(H) || std::memcmp(H.magic, kMagic, sizeof kMagic) != 0) {
    set_err("lbm_load: %s is not a saved subdomain state", path);
    return LBM_EINVAL;
  }
  const Header mine = header_of(h);
  if (std::memcmp(&H, &mine, sizeof H) != 0) {
    set_err("lbm_load: %s holds the state of another subdomain (size, node classes or "
            "parameters differ)", path);
    return LBM_EINVAL;
  }
  if (!F.get(rho_in) || !F.get(steps_done) || !get_ramp(F, R) || !F.get(nbuf) ||
      !(nbuf == 1 || nbuf == 3) || !finite_pos(rho_in)) {
    set_err("lbm_load: %s is truncated or corrupt", path);
    return LBM_EINVAL;
  }
  // a ramp in progress must carry settings lbm_drain_begin would accept
  if (R.phase != HostRamp::kIdle &&
      (check_drain_args(h, R.pc.data(), (int)R.pc.size(), &R.c, "lbm_load") != LBM_OK ||
       !(R.phase == HostRamp::kDone || R.point < (int)R.pc.size()))) {
    set_err("lbm_load: %s holds a drainage ramp with invalid settings (corrupt file)", path);
    return LBM_EINVAL;
  }
  if ((nbuf == 3) != (R.phase == HostRamp::kRamp || R.phase == HostRamp::kBisect)) {
    set_err("lbm_load: %s is truncated or corrupt", path);
    return LBM_EINVAL;
  }
  if (nbuf == 3) TRY(ensure_checkpoints(h, "lbm_load"));
  // from here on the handle's state is overwritten
  const size_t n = sc::pop_elems(h->nx, h->ny, h->nz);
  TRY(buffer_in(h, F, h->g[h->cur], n));
  if (nbuf == 3) {
    TRY(buffer_in(h, F, h->save[0], n));
    TRY(buffer_in(h, F, h->save[1], n));
  }
  TRY(set_rho_in(h, rho_in));
  h->steps_done = steps_done;
  h->ramp = std::move(R);
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_time_steps(lbm_throat_t h, long long nsteps, double *ms) {
  if (!h || nsteps < 0 || !ms) {
    set_err("lbm_time_steps: bad argument");
    return LBM_EINVAL;
  }
  HIPCHK(hipEventRecord(h->ev[0], h->stream));
  TRY(run_steps(h, nsteps));
  HIPCHK(hipEventRecord(h->ev[1], h->stream));
  HIPCHK(hipEventSynchronize(h->ev[1]));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, h->ev[0], h->ev[1]));
  *ms = t;
  return LBM_OK;
}

int lbm_step_timer(lbm_throat_t h, int enable, double *total_ms, long long *launches) {
  if (!h) {
    set_err("NULL handle");
    return LBM_EINVAL;
  }
  if (total_ms) *total_ms = h->timed_ms;
  if (launches) *launches = h->timed_launches;
  if (enable >= 0) {
    h->timing = enable != 0;
    h->timed_ms = 0.0;
    h->timed_launches = 0;
  }
  return LBM_OK;
}

int lbm_set_schedule(lbm_throat_t h, int tx, int ty, int lz) {
  if (!h) {
    set_err("NULL handle");
    return LBM_EINVAL;
  }
  sc::Sched s = h->sched;
  if (tx == sc::kListTx) {
    s = sc::Sched{sc::kListTx, 0, 0};
  } else {
    if (s.tx == sc::kListTx) s = sc::Sched{64, 4, 16};
    if (tx) s.tx = tx;
    if (ty) s.ty = ty;
    if (lz) s.lz = lz;
  }
  if (!sc::schedule_valid(s)) {
    set_err("schedule (%d, %d, %d) not supported", s.tx, s.ty, s.lz);
    return LBM_EINVAL;
  }
  h->sched = s;
  return rebuild_tiles(h);
}

int lbm_autotune(lbm_throat_t h, int trial_steps, int *tx, int *ty, int *lz) {
  if (!h || trial_steps < 1) {
    set_err("lbm_autotune: bad handle or trial_steps < 1");
    return LBM_EINVAL;
  }
  // Trials advance the state with alternating buffers, as the ramp does (a
  // trial that re-reads one unchanged buffer times some shapes faster than
  // they run), from a copy of g[cur] that is put back at the end, also on an
  // error path.  Every candidate runs an even number of steps, so the newest
  // state stays in g[cur].  The close candidates are timed a second time and
  // keep their faster time, so that a slow first pass (clocks, caches) does
  // not decide between shapes a few per cent apart.
  struct Keep {
    lbm_throat *h;
    float *d = nullptr;
    size_t bytes = 0;
    ~Keep() {
      if (!d) return;
      (void)hipMemcpyAsync(h->g[h->cur], d, bytes, hipMemcpyDeviceToDevice, h->stream);
      (void)hipStreamSynchronize(h->stream);
      (void)hipFree(d);
    }
  } keep{h};
  keep.bytes = sizeof(float) * sc::pop_elems(h->nx, h->ny, h->nz);
  if (hipMalloc((void **)&keep.d, keep.bytes) != hipSuccess) {
    keep.d = nullptr;
    set_err("lbm_autotune: hipMalloc of %zu bytes for the state copy failed", keep.bytes);
    return LBM_ENOMEM;
  }
  HIPCHK(hipMemcpyAsync(keep.d, h->g[h->cur], keep.bytes, hipMemcpyDeviceToDevice, h->stream));
  static const int lzs[7] = {1, 2, 4, 8, 16, 32, 64};
  std::vector<sc::Sched> cand;
  for (const auto &sh : sc::kShapes)
    for (int l : lzs)
      if (l <= h->nz) cand.push_back(sc::Sched{sh[0], sh[1], l});
  cand.push_back(sc::Sched{sc::kListTx, 0, 0});
  std::vector<double> t(cand.size(), INFINITY);
  auto trial = [&](size_t c) -> int {
    const sc::Sched &s = cand[c];
    h->sched = s;
    TRY(rebuild_tiles(h));
    int par = h->cur;
    auto one = [&]() {
      const hipError_t e = sc::launch_step(h->desc_d, h->tiles_d, h->ntiles, s.tx, s.ty, par,
                                           h->stream, h->zper_d, h->n_zper);
      par ^= 1;
      return e;
    };
    for (int w = 0; w < 2; ++w) HIPCHK(one());
    HIPCHK(hipEventRecord(h->ev[0], h->stream));
    for (int i = 0; i < trial_steps; ++i) HIPCHK(one());
    HIPCHK(hipEventRecord(h->ev[1], h->stream));
    if (trial_steps & 1) HIPCHK(one());
    HIPCHK(hipEventSynchronize(h->ev[1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
    t[c] = std::min(t[c], (double)ms);
    return LBM_OK;
  };
  // first round: per tile shape in increasing lz, stop once a segment length
  // is 1.5x slower than the shape's best (longer ones only lengthen the
  // serial z-march); second round: the candidates within 1.25x of the best
  for (size_t c = 0; c < cand.size();) {
    double shape_best = INFINITY;
    size_t e = c;
    while (e < cand.size() && cand[e].tx == cand[c].tx && cand[e].ty == cand[c].ty) ++e;
    for (size_t k = c; k < e; ++k) {
      TRY(trial(k));
      if (t[k] > 1.5 * shape_best) break;
      shape_best = std::min(shape_best, t[k]);
    }
    c = e;
  }
  const double first = *std::min_element(t.begin(), t.end());
  for (size_t c = 0; c < cand.size(); ++c)
    if (t[c] <= 1.25 * first) TRY(trial(c));
  size_t best = 0;
  for (size_t c = 1; c < cand.size(); ++c)
    if (t[c] < t[best]) best = c;
  h->sched = cand[best];
  TRY(rebuild_tiles(h));
  if (tx) *tx = h->sched.tx;
  if (ty) *ty = h->sched.ty;
  if (lz) *lz = h->sched.lz;
  return LBM_OK;
}

int lbm_place(lbm_throat_t h, int tries, int trial_steps, double *ms_first, double *ms_best) {
  if (!h || tries < 0 || tries > 8 || trial_steps < 1) {
    set_err("lbm_place: bad handle, tries outside 0..8 or trial_steps < 1");
    return LBM_EINVAL;
  }
  const size_t bytes = sizeof(float) * sc::pop_elems(h->nx, h->ny, h->nz);
  TRY(lbmh::check_budget(bytes * (1 + 2 * (size_t)tries), "lbm_place"));
  // The state is kept in a copy; each placement (the current pair, then
  // `tries` new pairs allocated while the earlier ones are still held, so
  // that they land elsewhere) runs 2 + trial_steps steps from that copy with
  // alternating buffers, timed with events; the fastest pair gets the copy
  // back and the others are freed, also on an error path.
  struct Pair {
    float *g[2] = {nullptr, nullptr};
  };
  struct Work {
    lbm_throat *h;
    float *keep = nullptr;
    size_t bytes = 0;
    Pair orig;
    std::vector<Pair> cand;
    int chosen = -1;  // -1: the original pair
    ~Work() {
      // the handle keeps the chosen pair; the copy goes back into it
      if (chosen >= 0) {
        h->g[0] = cand[chosen].g[0];
        h->g[1] = cand[chosen].g[1];
        h->cur = 0;
      } else {
        h->g[0] = orig.g[0];
        h->g[1] = orig.g[1];
      }
      if (keep)
        (void)hipMemcpyAsync(h->g[h->cur], keep, bytes, hipMemcpyDeviceToDevice, h->stream);
      (void)sync_desc(h);
      (void)hipStreamSynchronize(h->stream);
      for (int i = 0; i < (int)cand.size(); ++i)
        if (i != chosen)
          for (float *b : cand[i].g)
            if (b) (void)hipFree(b);
      if (chosen >= 0)
        for (float *b : orig.g) (void)hipFree(b);
      if (keep) (void)hipFree(keep);
    }
  } w{h};
  w.bytes = bytes;
  w.orig.g[0] = h->g[0];
  w.orig.g[1] = h->g[1];
  if (hipMalloc((void **)&w.keep, bytes) != hipSuccess) {
    w.keep = nullptr;
    set_err("lbm_place: hipMalloc of %zu bytes for the state copy failed", bytes);
    return LBM_ENOMEM;
  }
  HIPCHK(hipMemcpyAsync(w.keep, h->g[h->cur], bytes, hipMemcpyDeviceToDevice, h->stream));
  const int state0 = h->cur;
  auto timed = [&](const Pair &pr, int parity, double *ms) -> int {
    h->g[0] = pr.g[0];
    h->g[1] = pr.g[1];
    TRY(sync_desc(h));
    HIPCHK(hipMemcpyAsync(pr.g[parity], w.keep, bytes, hipMemcpyDeviceToDevice, h->stream));
    int par = parity;
    auto one = [&]() {
      const hipError_t e = sc::launch_step(h->desc_d, h->tiles_d, h->ntiles, h->sched.tx,
                                           h->sched.ty, par, h->stream, h->zper_d, h->n_zper);
      par ^= 1;
      return e;
    };
    for (int i = 0; i < 2; ++i) HIPCHK(one());
    HIPCHK(hipEventRecord(h->ev[0], h->stream));
    for (int i = 0; i < trial_steps; ++i) HIPCHK(one());
    HIPCHK(hipEventRecord(h->ev[1], h->stream));
    HIPCHK(hipEventSynchronize(h->ev[1]));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, h->ev[0], h->ev[1]));
    *ms = (double)t / trial_steps;
    return LBM_OK;
  };
  double best = 0.0;
  TRY(timed(w.orig, state0, &best));
  const double first = best;
  for (int k = 0; k < tries; ++k) {
    Pair pr;
    if (hipMalloc((void **)&pr.g[0], bytes) != hipSuccess ||
        hipMalloc((void **)&pr.g[1], bytes) != hipSuccess) {
      (void)hipGetLastError();
      if (pr.g[0]) (void)hipFree(pr.g[0]);
      break;  // no room for another placement: keep the best so far
    }
    w.cand.push_back(pr);
    double t = 0.0;
    TRY(timed(pr, 0, &t));
    if (t < best) {
      best = t;
      w.chosen = (int)w.cand.size() - 1;
    }
  }
  if (w.chosen < 0) h->cur = state0;
  if (ms_first) *ms_first = first;
  if (ms_best) *ms_best = best;
  return LBM_OK;
}

int lbm_get_schedule(lbm_throat_t h, int *tx, int *ty, int *lz) {
  if (!h) {
    set_err("NULL handle");
    return LBM_EINVAL;
  }
  if (tx) *tx = h->sched.tx;
  if (ty) *ty = h->sched.ty;
  if (lz) *lz = h->sched.lz;
  return LBM_OK;
}

int lbm_bw_probe(size_t bytes, int reps, double *gbps) {
  if (bytes < (1u << 20) || reps < 1 || !gbps) {
    set_err("lbm_bw_probe: bytes >= 1 MiB, reps >= 1 and an output are required");
    return LBM_EINVAL;
  }
  const size_t nf = bytes / 16 * 4;
  float *a = nullptr, *b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  if (hipMalloc((void **)&a, nf * sizeof(float)) != hipSuccess ||
      hipMalloc((void **)&b, nf * sizeof(float)) != hipSuccess) {
    set_err("lbm_bw_probe: hipMalloc of 2 x %zu bytes failed", nf * sizeof(float));
    rc = LBM_ENOMEM;
  }
  if (rc == LBM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
                       hipMemset(a, 0, nf * sizeof(float)) != hipSuccess)) {
    set_err("lbm_bw_probe: setup failed");
    rc = LBM_EHIP;
  }
  if (rc == LBM_OK) {
    hipError_t e = sc::launch_copy(a, b, nf, nullptr);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = sc::launch_copy(a, b, nf, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      set_err("lbm_bw_probe: %s", hipGetErrorString(e));
      rc = LBM_EHIP;
    } else {
      *gbps = 2.0 * (double)nf * sizeof(float) * reps / (ms * 1e-3) / 1e9;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}

}  // extern "C"
