// surrogate.cpp -- C ABI of the learned entry-pressure surrogate
// (lbm_surrogate.h): an ensemble of MLPs trained on the GPU with BF16
// matrix-core products, used to answer throats whose members agree and to
// hand the others to the batched LBM drainage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lbm_abi.h"
#include "lbm_handle.h"
#include "lbm_surrogate.h"
#include "sg_internal.h"

using lbmh::set_err;

#define SGCHK(call)                                                           \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_err("%s failed: %s", #call, hipGetErrorString(e_));                 \
      return LBM_EHIP;                                                        \
    }                                                                         \
  } while (0)

#define SGTRY(call)                                                           \
  do {                                                                        \
    int r_ = (call);                                                          \
    if (r_ != LBM_OK) return r_;                                              \
  } while (0)

static_assert(sg::kParams == LBM_SG_NPARAM, "parameter count");
static_assert(sg::kFeat == LBM_SG_NFEAT && sg::kOut == LBM_SG_NOUT, "widths");

namespace {

constexpr long long P = sg::kParams;
constexpr int H = sg::kHidden;

uint64_t splitmix64(uint64_t seed, uint64_t i) {
  // i-th output (i >= 0) of SplitMix64 seeded with seed, counter style
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double u01(uint64_t seed, uint64_t i) { return (double)(splitmix64(seed, i) >> 11) * 0x1.0p-53; }

template <class T>
int dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return LBM_OK;
  if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_err("hipMalloc of %zu bytes failed", count * sizeof(T));
    return LBM_ENOMEM;
  }
  return LBM_OK;
}

template <class T>
void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

struct lbm_surrogate {
  int members = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // [members][P]
  sg::bf16 *wb = nullptr;
  long long adam_t = 0;
  bool has_stats = false;
  double *stats_d = nullptr;  // xmu[80] xsd[80] tmu[17] tsd[17]
  double *loss_d = nullptr;   // [members]
  // work buffers of batch capacity cap
  int cap = 0;
  sg::bf16 *act[4] = {};  // bf16 layer inputs [members][cap][width]
  float *zpre[3] = {};    // hidden pre-activations [members][cap][256]
  float *dz[3] = {};      // their gradients, f32 and bf16
  sg::bf16 *dzb[3] = {};
  float *y = nullptr, *t = nullptr, *dy = nullptr;  // [members][cap][17]
  sg::bf16 *dyb = nullptr;
  hipEvent_t ev[2] = {};

  double *xmu() { return stats_d; }
  double *xsd() { return stats_d + 80; }
  double *tmu() { return stats_d + 160; }
  double *tsd() { return stats_d + 177; }

  void free_work() {
    for (auto &p : act) dfree(p);
    for (auto &p : zpre) dfree(p);
    for (auto &p : dz) dfree(p);
    for (auto &p : dzb) dfree(p);
    dfree(y);
    dfree(t);
    dfree(dy);
    dfree(dyb);
    cap = 0;
  }

  int ensure(int need) {
    if (need <= cap) return LBM_OK;
    if (hipStreamSynchronize(stream) != hipSuccess) {
      set_err("stream synchronisation failed");
      return LBM_EHIP;
    }
    free_work();
    const size_t M = (size_t)members, c = (size_t)need;
    SGTRY(dalloc(&act[0], M * c * sg::kFeat));
    for (int l = 1; l < 4; ++l) SGTRY(dalloc(&act[l], M * c * H));
    for (int l = 0; l < 3; ++l) {
      SGTRY(dalloc(&zpre[l], M * c * H));
      SGTRY(dalloc(&dz[l], M * c * H));
      SGTRY(dalloc(&dzb[l], M * c * H));
    }
    SGTRY(dalloc(&y, M * c * sg::kOut));
    SGTRY(dalloc(&t, M * c * sg::kOut));
    SGTRY(dalloc(&dy, M * c * sg::kOut));
    SGTRY(dalloc(&dyb, M * c * sg::kOut));
    cap = need;
    return LBM_OK;
  }

  ~lbm_surrogate() {
    if (stream) (void)hipStreamSynchronize(stream);
    free_work();
    dfree(w);
    dfree(m);
    dfree(v);
    dfree(g);
    dfree(wb);
    dfree(stats_d);
    dfree(loss_d);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  // forward of a batch already in act[0]; saz0 = 0 shares one input among
  // the members
  int forward(int bsz, long long saz0) {
    const long long c = cap;
    for (int l = 0; l < 4; ++l) {
      const int K = sg::kWidth[l], N = sg::kWidth[l + 1];
      sg::Gemm q{};
      q.A = act[l];
      q.sam = K;
      q.sak = 1;
      q.saz = l == 0 ? saz0 : c * K;
      q.B = wb + sg::w_off(l);  // B(k, n) = W[n][k]
      q.sbk = 1;
      q.sbn = K;
      q.sbz = P;
      q.M = bsz;
      q.N = N;
      q.K = K;
      q.members = members;
      q.bias = w + sg::b_off(l);
      q.bstride = P;
      if (l < 3) {
        q.epi = sg::kEpiBiasSilu;
        q.C = zpre[l];
        q.scz = c * N;
        q.Cb = act[l + 1];
        q.sbzc = c * N;
      } else {
        q.epi = sg::kEpiBiasF32;
        q.C = y;
        q.scz = c * N;
      }
      SGCHK(sg::launch_gemm(q, stream));
    }
    return LBM_OK;
  }

  // gradients of the loss into g after forward(); targets in t
  int backward(int bsz) {
    const long long c = cap;
    SGCHK(sg::launch_loss_grad(y, t, members, bsz, c, dy, dyb, loss_d, stream));
    for (int l = 3; l >= 0; --l) {
      const int K = sg::kWidth[l], N = sg::kWidth[l + 1];
      const sg::bf16 *Db = l == 3 ? dyb : dzb[l];
      const float *Df = l == 3 ? dy : dz[l];
      // dW[n][k] = sum_b D[b][n] act[b][k]
      sg::Gemm q{};
      q.A = Db;
      q.sam = 1;
      q.sak = N;
      q.saz = c * N;
      q.B = act[l];
      q.sbk = K;
      q.sbn = 1;
      q.sbz = c * K;
      q.M = N;
      q.N = K;
      q.K = bsz;
      q.members = members;
      q.epi = sg::kEpiF32;
      q.C = g + sg::w_off(l);
      q.scz = P;
      SGCHK(sg::launch_gemm(q, stream));
      SGCHK(sg::launch_bias_grad(Df, members, bsz, N, c, g + sg::b_off(l), P, stream));
      if (l == 0) break;
      // d act[b][k] = sum_n D[b][n] W[n][k], times silu'(z) of the layer below
      sg::Gemm r{};
      r.A = Db;
      r.sam = N;
      r.sak = 1;
      r.saz = c * N;
      r.B = wb + sg::w_off(l);
      r.sbk = K;
      r.sbn = 1;
      r.sbz = P;
      r.M = bsz;
      r.N = K;
      r.K = N;
      r.members = members;
      r.epi = sg::kEpiDsilu;
      r.Zin = zpre[l - 1];
      r.szz = c * K;
      r.C = dz[l - 1];
      r.scz = c * K;
      r.Cb = dzb[l - 1];
      r.sbzc = c * K;
      SGCHK(sg::launch_gemm(r, stream));
    }
    return LBM_OK;
  }
};

namespace {

int check_model(lbm_surrogate_t s) {
  if (!s) {
    set_err("surrogate handle is NULL");
    return LBM_EINVAL;
  }
  return LBM_OK;
}

bool all_finite(const double *a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// upload host doubles [n][cols] into a scratch device array and standardise
// with (mu, sd) into f32
int upload_std(lbm_surrogate_t s, const double *host, int n, int cols, const double *mu,
               const double *sd, float **out) {
  double *tmp = nullptr;
  SGTRY(dalloc(&tmp, (size_t)n * cols));
  if (int r = dalloc(out, (size_t)n * cols)) {
    dfree(tmp);
    return r;
  }
  hipError_t e = hipMemcpyAsync(tmp, host, sizeof(double) * n * cols, hipMemcpyHostToDevice,
                                s->stream);
  if (e == hipSuccess) e = sg::launch_standardise(tmp, n, cols, mu, sd, *out, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  dfree(tmp);
  if (e != hipSuccess) {
    dfree(*out);
    set_err("standardising inputs failed: %s", hipGetErrorString(e));
    return LBM_EHIP;
  }
  return LBM_OK;
}

// device arrays of zeros / ones for "no standardisation"
struct Identity {
  double *zero = nullptr, *one = nullptr;
  int make(hipStream_t st) {
    std::vector<double> z(sg::kFeat, 0.0), o(sg::kFeat, 1.0);
    SGTRY(dalloc(&zero, z.size()));
    SGTRY(dalloc(&one, o.size()));
    SGCHK(hipMemcpyAsync(zero, z.data(), sizeof(double) * z.size(), hipMemcpyHostToDevice, st));
    SGCHK(hipMemcpyAsync(one, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice, st));
    return LBM_OK;
  }
  ~Identity() {
    dfree(zero);
    dfree(one);
  }
};

// forward of n standardised rows (device f32 [n][80]) in chunks; calls
// sink(start, count) after each chunk with the outputs in s->y
template <class F>
int forward_chunks(lbm_surrogate_t s, const float *xs_d, int n, F sink) {
  const int chunk = std::min(n, LBM_SG_MAX_BATCH);
  SGTRY(s->ensure(chunk));
  for (int start = 0; start < n; start += chunk) {
    const int cnt = std::min(chunk, n - start);
    SGCHK(sg::launch_gather(xs_d + (size_t)start * sg::kFeat, nullptr, nullptr, 0, 1, cnt, s->cap,
                            s->act[0], nullptr, s->stream));
    SGTRY(s->forward(cnt, 0));
    SGTRY(sink(start, cnt));
  }
  return LBM_OK;
}

// Mayer-Stowe-Princen entry radius of the throat's cross-section (Sec. 1 of
// the paper names the method): the triangle of the three throat-sphere
// centres (the prism's walls run along its edges) minus the three circles.
// With corner menisci of radius r the wetting phase holds, per edge: where
// the circles overlap or touch, the corner closed by the arc tangent to both;
// where they leave a gap, the two right-angled circle-wall corners, each
// closed by the arc tangent to its circle and the wall, or the whole gap once
// those two arcs would meet (closed by the arc tangent to both circles).  The
// non-wetting phase takes the rest, area A_n, bounded by the menisci (L_nw),
// the remaining circle arcs and the dry wall segments (L_ns); entry is the
// root of the force balance A_n = r (L_nw + L_ns) for a perfectly wetting
// solid, and p_c = gamma / r.
double half_lens(double a, double b, double d) {
  if (d >= a + b) return 0.0;
  const double ca = std::max(-1.0, std::min(1.0, (d * d + a * a - b * b) / (2.0 * d * a)));
  const double cb = std::max(-1.0, std::min(1.0, (d * d + b * b - a * a) / (2.0 * d * b)));
  const double k = std::max(0.0, (-d + a + b) * (d + a - b) * (d - a + b) * (d + a + b));
  return 0.5 * (a * a * std::acos(ca) + b * b * std::acos(cb) - 0.5 * std::sqrt(k));
}

double vertex_angle(const double *p, const double *q, const double *s) {
  const double u[2] = {q[0] - p[0], q[1] - p[1]}, v[2] = {s[0] - p[0], s[1] - p[1]};
  const double c = (u[0] * v[0] + u[1] * v[1]) / (std::hypot(u[0], u[1]) * std::hypot(v[0], v[1]));
  return std::acos(std::max(-1.0, std::min(1.0, c)));
}

struct Section {
  double C[3][2], R[3];
};

// (A_n, L_nw + L_ns) for corner menisci of radius r; false when the menisci
// would overlap or leave no non-wetting area
bool msp_parts(const Section &S, double r, double &An, double &L) {
  const double pi = 3.14159265358979323846;
  double area = 0.5 * std::fabs((S.C[1][0] - S.C[0][0]) * (S.C[2][1] - S.C[0][1]) -
                                (S.C[2][0] - S.C[0][0]) * (S.C[1][1] - S.C[0][1]));
  double theta[3], used[3] = {0.0, 0.0, 0.0}, wet = 0.0;
  L = 0.0;
  for (int i = 0; i < 3; ++i) {
    const int j = (i + 1) % 3, k = (i + 2) % 3;
    theta[i] = vertex_angle(S.C[i], S.C[j], S.C[k]);
    const double d = std::hypot(S.C[j][0] - S.C[i][0], S.C[j][1] - S.C[i][1]);
    area += -0.5 * S.R[i] * S.R[i] * theta[i] + half_lens(S.R[i], S.R[j], d);
  }
  for (int i = 0; i < 3; ++i) {
    const int j = (i + 1) % 3;
    const double d = std::hypot(S.C[j][0] - S.C[i][0], S.C[j][1] - S.C[i][1]);
    if (S.R[i] + S.R[j] < d) {
      const double fi = std::sqrt((S.R[i] + r) * (S.R[i] + r) - r * r);
      const double fj = std::sqrt((S.R[j] + r) * (S.R[j] + r) - r * r);
      if (fi + fj <= d) {  // two circle-wall corners and a dry wall segment
        const double f2[2] = {fi, fj};
        const int q2[2] = {i, j};
        for (int e = 0; e < 2; ++e) {
          const double g = std::atan2(r, f2[e]), Rq = S.R[q2[e]];
          wet += 0.5 * f2[e] * r - 0.5 * Rq * Rq * g - 0.5 * r * r * (0.5 * pi - g);
          L += r * (0.5 * pi - g);
          used[q2[e]] += g;
        }
        L += d - fi - fj;
        continue;
      }
    }
    // the corner (or the whole gap) closed by the arc tangent to both circles
    const double a = S.R[i] + r, b = S.R[j] + r;
    const double ai = std::acos(std::max(-1.0, std::min(1.0, (d * d + a * a - b * b) / (2.0 * d * a))));
    const double aj = std::acos(std::max(-1.0, std::min(1.0, (d * d + b * b - a * a) / (2.0 * d * b))));
    const double beta = pi - ai - aj;
    wet += 0.5 * d * a * std::sin(ai) - 0.5 * S.R[i] * S.R[i] * ai - 0.5 * S.R[j] * S.R[j] * aj -
           0.5 * r * r * beta + half_lens(S.R[i], S.R[j], d);
    L += r * beta;
    used[i] += ai;
    used[j] += aj;
  }
  bool valid = true;
  for (int i = 0; i < 3; ++i) {
    const double rest = theta[i] - used[i];
    valid = valid && rest >= 0.0;
    L += S.R[i] * std::max(rest, 0.0);
  }
  An = area - wet;
  return valid && An > 0.0;
}

// MS-P corner-meniscus radius at entry of the throat whose three spheres are
// G[0..11] (x, y, z, R each; the cross-section is the xy-plane), or NaN where
// no root lies in the range of valid radii: scan r upward by factors of 1.15
// from 1e-6 of the largest radius until the balance changes sign, then bisect
// the bracket to 1e-13 of that radius.
double msp_radius(const double *G) {
  Section S;
  double scale = 0.0;
  for (int i = 0; i < 3; ++i) {
    S.C[i][0] = G[4 * i];
    S.C[i][1] = G[4 * i + 1];
    S.R[i] = G[4 * i + 3];
    scale = std::max(scale, S.R[i]);
  }
  // (the scan starts at a positive radius and ends above 10x the scale, so
  // it needs a positive, finite scale to terminate)
  if (!(scale > 0.0 && scale < INFINITY)) return NAN;
  auto f = [&](double r) {
    double An, L;
    msp_parts(S, r, An, L);
    return An - r * L;
  };
  double r = 1e-6 * scale;
  if (!(f(r) > 0.0)) return NAN;
  for (;;) {
    const double nxt = r * 1.15;
    double An, L;
    if (!msp_parts(S, nxt, An, L)) return NAN;
    if (An - nxt * L < 0.0) {
      double lo = r, hi = nxt;
      while (hi - lo > 1e-13 * scale) {
        const double mid = 0.5 * (lo + hi);
        (f(mid) > 0.0 ? lo : hi) = mid;
      }
      return 0.5 * (lo + hi);
    }
    r = nxt;
    if (r > 10.0 * scale) return NAN;
  }
}

int params_geometry(int n, const lbm_params *p, std::vector<double> &geo) {
  geo.assign((size_t)n * 19, 0.0);
  for (int t = 0; t < n; ++t) {
    const lbm_params &q = p[t];
    if (q.n_spheres != 4 || !q.spheres || !q.prism) {
      set_err("throat %d: the descriptor needs exactly 4 spheres and a prism closure", t);
      return LBM_EINVAL;
    }
    int ids[4] = {q.prism_ids[0], q.prism_ids[1], q.prism_ids[2], -1};
    for (int i = 0; i < 4; ++i)
      if (i != ids[0] && i != ids[1] && i != ids[2]) ids[3] = i;
    if (ids[3] < 0 || ids[0] == ids[1] || ids[1] == ids[2] || ids[0] == ids[2]) {
      set_err("throat %d: prism_ids must name three distinct spheres of 0..3", t);
      return LBM_EINVAL;
    }
    double *G = geo.data() + (size_t)t * 19;
    for (int i = 0; i < 4; ++i) {
      const lbm_sphere &sp = q.spheres[ids[i]];
      if (!(std::isfinite(sp.c[0]) && std::isfinite(sp.c[1]) && std::isfinite(sp.c[2]) &&
            std::isfinite(sp.r) && sp.r > 0)) {
        set_err("throat %d: sphere %d has a non-finite centre or a non-positive radius", t,
                ids[i]);
        return LBM_EINVAL;
      }
      G[4 * i + 0] = sp.c[0];
      G[4 * i + 1] = sp.c[1];
      G[4 * i + 2] = sp.c[2];
      G[4 * i + 3] = sp.r;
    }
    G[16] = q.nx;
    G[17] = q.ny;
    G[18] = q.nz;
    if (!all_finite(G, 19) || !(G[3] > 0 && G[7] > 0 && G[11] > 0 && G[15] > 0)) {
      set_err("throat %d: sphere data must be finite with positive radii", t);
      return LBM_EINVAL;
    }
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_surrogate_create(int members, unsigned long long seed, void *stream,
                         lbm_surrogate_t *out) {
  if (!out || members < 1 || members > LBM_SG_MAX_MEMBERS) {
    set_err("lbm_surrogate_create: members must be 1..%d and out non-NULL", LBM_SG_MAX_MEMBERS);
    return LBM_EINVAL;
  }
  *out = nullptr;
  lbm_surrogate *s = new lbm_surrogate();
  s->members = members;
  auto fail = [&](int r) {
    delete s;
    return r;
  };
  if (stream) {
    s->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&s->stream) != hipSuccess) {
      set_err("hipStreamCreate failed");
      return fail(LBM_EHIP);
    }
    s->own_stream = true;
  }
  const size_t count = (size_t)members * P;
  if (int r = dalloc(&s->w, count)) return fail(r);
  if (int r = dalloc(&s->m, count)) return fail(r);
  if (int r = dalloc(&s->v, count)) return fail(r);
  if (int r = dalloc(&s->g, count)) return fail(r);
  if (int r = dalloc(&s->wb, count)) return fail(r);
  if (int r = dalloc(&s->stats_d, 194)) return fail(r);
  if (int r = dalloc(&s->loss_d, (size_t)members)) return fail(r);
  for (auto &e : s->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      set_err("hipEventCreate failed");
      return fail(LBM_EHIP);
    }
  std::vector<float> h((size_t)P);
  for (int z = 0; z < members; ++z) {
    const uint64_t sd = splitmix64(seed, (uint64_t)z);
    uint64_t i = 0;
    std::fill(h.begin(), h.end(), 0.f);
    for (int l = 0; l < sg::kLayers; ++l) {
      const int K = sg::kWidth[l], N = sg::kWidth[l + 1];
      const double a = std::sqrt(3.0 / K);
      float *W = h.data() + sg::w_off(l);
      for (long long j = 0; j < (long long)N * K; ++j) W[j] = (float)(a * (2.0 * u01(sd, i++) - 1.0));
    }
    if (hipMemcpy(s->w + (size_t)z * P, h.data(), sizeof(float) * P, hipMemcpyHostToDevice) !=
        hipSuccess) {
      set_err("weight upload failed");
      return fail(LBM_EHIP);
    }
  }
  if (hipMemset(s->m, 0, sizeof(float) * count) != hipSuccess ||
      hipMemset(s->v, 0, sizeof(float) * count) != hipSuccess ||
      sg::launch_to_bf16(s->w, s->wb, (long long)count, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess) {
    set_err("model initialisation failed");
    return fail(LBM_EHIP);
  }
  *out = s;
  return LBM_OK;
}

void lbm_surrogate_free(lbm_surrogate_t s) { delete s; }

int lbm_surrogate_members(lbm_surrogate_t s) { return s ? s->members : 0; }

int lbm_surrogate_set_params(lbm_surrogate_t s, int member, const float *w) {
  SGTRY(check_model(s));
  if (member < 0 || member >= s->members || !w) {
    set_err("lbm_surrogate_set_params: member out of range or NULL array");
    return LBM_EINVAL;
  }
  for (long long i = 0; i < P; ++i)
    if (!std::isfinite(w[i])) {
      set_err("lbm_surrogate_set_params: parameter %lld is not finite", i);
      return LBM_ENONFINITE;
    }
  float *dst = s->w + (size_t)member * P;
  SGCHK(hipMemcpyAsync(dst, w, sizeof(float) * P, hipMemcpyHostToDevice, s->stream));
  SGCHK(hipMemsetAsync(s->m + (size_t)member * P, 0, sizeof(float) * P, s->stream));
  SGCHK(hipMemsetAsync(s->v + (size_t)member * P, 0, sizeof(float) * P, s->stream));
  SGCHK(sg::launch_to_bf16(dst, s->wb + (size_t)member * P, P, s->stream));
  SGCHK(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

int lbm_surrogate_get_params(lbm_surrogate_t s, int member, float *w) {
  SGTRY(check_model(s));
  if (member < 0 || member >= s->members || !w) {
    set_err("lbm_surrogate_get_params: member out of range or NULL array");
    return LBM_EINVAL;
  }
  SGCHK(hipMemcpyAsync(w, s->w + (size_t)member * P, sizeof(float) * P, hipMemcpyDeviceToHost,
                       s->stream));
  SGCHK(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

int lbm_surrogate_set_stats(lbm_surrogate_t s, const double *xmu, const double *xsd,
                            const double *tmu, const double *tsd) {
  SGTRY(check_model(s));
  if (!xmu || !xsd || !tmu || !tsd) {
    set_err("lbm_surrogate_set_stats: NULL array");
    return LBM_EINVAL;
  }
  double h[194];
  std::memcpy(h, xmu, sizeof(double) * 80);
  std::memcpy(h + 80, xsd, sizeof(double) * 80);
  std::memcpy(h + 160, tmu, sizeof(double) * 17);
  std::memcpy(h + 177, tsd, sizeof(double) * 17);
  if (!all_finite(h, 194)) {
    set_err("lbm_surrogate_set_stats: values must be finite");
    return LBM_ENONFINITE;
  }
  for (int i = 0; i < 80; ++i)
    if (!(h[80 + i] > 0)) {
      set_err("lbm_surrogate_set_stats: standard deviations must be > 0");
      return LBM_EINVAL;
    }
  for (int i = 0; i < 17; ++i)
    if (!(h[177 + i] > 0)) {
      set_err("lbm_surrogate_set_stats: standard deviations must be > 0");
      return LBM_EINVAL;
    }
  SGCHK(hipMemcpyAsync(s->stats_d, h, sizeof h, hipMemcpyHostToDevice, s->stream));
  SGCHK(hipStreamSynchronize(s->stream));
  s->has_stats = true;
  return LBM_OK;
}

int lbm_surrogate_get_stats(lbm_surrogate_t s, double *xmu, double *xsd, double *tmu,
                            double *tsd) {
  SGTRY(check_model(s));
  if (!s->has_stats) {
    set_err("lbm_surrogate_get_stats: the model has no statistics yet");
    return LBM_ESTATE;
  }
  if (!xmu || !xsd || !tmu || !tsd) {
    set_err("lbm_surrogate_get_stats: NULL array");
    return LBM_EINVAL;
  }
  double h[194];
  SGCHK(hipMemcpyAsync(h, s->stats_d, sizeof h, hipMemcpyDeviceToHost, s->stream));
  SGCHK(hipStreamSynchronize(s->stream));
  std::memcpy(xmu, h, sizeof(double) * 80);
  std::memcpy(xsd, h + 80, sizeof(double) * 80);
  std::memcpy(tmu, h + 160, sizeof(double) * 17);
  std::memcpy(tsd, h + 177, sizeof(double) * 17);
  return LBM_OK;
}

int lbm_surrogate_describe(int n, const lbm_params *p, double *feat, double *r_msp) {
  if (n < 0 || (n > 0 && (!p || !feat))) {
    set_err("lbm_surrogate_describe: bad arguments");
    return LBM_EINVAL;
  }
  if (n == 0) return LBM_OK;
  std::vector<double> geo;
  SGTRY(params_geometry(n, p, geo));
  if (r_msp)
    for (int t = 0; t < n; ++t) r_msp[t] = msp_radius(geo.data() + (size_t)t * 19);
  hipStream_t st = (hipStream_t)p[0].stream;
  double *geo_d = nullptr, *feat_d = nullptr;
  SGTRY(dalloc(&geo_d, geo.size()));
  if (int r = dalloc(&feat_d, (size_t)n * sg::kFeat)) {
    dfree(geo_d);
    return r;
  }
  hipError_t e = hipMemcpyAsync(geo_d, geo.data(), sizeof(double) * geo.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = sg::launch_describe(geo_d, n, feat_d, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(feat, feat_d, sizeof(double) * n * sg::kFeat, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(geo_d);
  dfree(feat_d);
  if (e != hipSuccess) {
    set_err("lbm_surrogate_describe: %s", hipGetErrorString(e));
    return LBM_EHIP;
  }
  return LBM_OK;
}

int lbm_surrogate_forward(lbm_surrogate_t s, int n, const double *xs, float *y) {
  SGTRY(check_model(s));
  if (n < 0 || (n > 0 && (!xs || !y))) {
    set_err("lbm_surrogate_forward: bad arguments");
    return LBM_EINVAL;
  }
  if (n == 0) return LBM_OK;
  if (!all_finite(xs, (size_t)n * sg::kFeat)) {
    set_err("lbm_surrogate_forward: inputs must be finite");
    return LBM_ENONFINITE;
  }
  Identity id;
  SGTRY(id.make(s->stream));
  float *xs_d = nullptr;
  SGTRY(upload_std(s, xs, n, sg::kFeat, id.zero, id.one, &xs_d));
  int rc = forward_chunks(s, xs_d, n, [&](int start, int cnt) -> int {
    for (int z = 0; z < s->members; ++z)
      SGCHK(hipMemcpyAsync(y + ((size_t)z * n + start) * sg::kOut,
                           s->y + (size_t)z * s->cap * sg::kOut, sizeof(float) * cnt * sg::kOut,
                           hipMemcpyDeviceToHost, s->stream));
    SGCHK(hipStreamSynchronize(s->stream));
    return LBM_OK;
  });
  dfree(xs_d);
  return rc;
}

int lbm_surrogate_grad(lbm_surrogate_t s, int n, const double *xs, const double *ts, float *grad,
                       double *loss) {
  SGTRY(check_model(s));
  if (n < 1 || n > LBM_SG_MAX_BATCH || !xs || !ts || !grad) {
    set_err("lbm_surrogate_grad: need 1 <= n <= %d and non-NULL arrays", LBM_SG_MAX_BATCH);
    return LBM_EINVAL;
  }
  if (!all_finite(xs, (size_t)n * sg::kFeat) || !all_finite(ts, (size_t)n * sg::kOut)) {
    set_err("lbm_surrogate_grad: inputs must be finite");
    return LBM_ENONFINITE;
  }
  Identity id;
  SGTRY(id.make(s->stream));
  float *xs_d = nullptr, *ts_d = nullptr;
  SGTRY(upload_std(s, xs, n, sg::kFeat, id.zero, id.one, &xs_d));
  if (int r = upload_std(s, ts, n, sg::kOut, id.zero, id.one, &ts_d)) {
    dfree(xs_d);
    return r;
  }
  int rc = s->ensure(n);
  if (rc == LBM_OK) {
    hipError_t e = sg::launch_gather(xs_d, ts_d, nullptr, 0, s->members, n, s->cap, s->act[0],
                                     s->t, s->stream);
    if (e != hipSuccess) {
      set_err("gather failed: %s", hipGetErrorString(e));
      rc = LBM_EHIP;
    }
  }
  if (rc == LBM_OK) rc = s->forward(n, (long long)s->cap * sg::kFeat);
  if (rc == LBM_OK) rc = s->backward(n);
  if (rc == LBM_OK) {
    hipError_t e = hipMemcpyAsync(grad, s->g, sizeof(float) * s->members * P,
                                  hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && loss)
      e = hipMemcpyAsync(loss, s->loss_d, sizeof(double) * s->members, hipMemcpyDeviceToHost,
                         s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
      set_err("lbm_surrogate_grad: %s", hipGetErrorString(e));
      rc = LBM_EHIP;
    }
  }
  dfree(xs_d);
  dfree(ts_d);
  return rc;
}

int lbm_surrogate_train(lbm_surrogate_t s, int n, const double *feat, const double *target,
                        const lbm_sg_train_cfg *cfg, const int *order, double *loss_hist) {
  SGTRY(check_model(s));
  if (n < 2 || !feat || !target || !cfg) {
    set_err("lbm_surrogate_train: need n >= 2 and non-NULL feat, target, cfg");
    return LBM_EINVAL;
  }
  if (cfg->epochs < 1 || cfg->batch < 1 || cfg->batch > LBM_SG_MAX_BATCH || !(cfg->lr > 0) ||
      !(cfg->lr_min_frac >= 0 && cfg->lr_min_frac <= 1) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) ||
      !(cfg->beta2 >= 0 && cfg->beta2 < 1) || !(cfg->eps > 0)) {
    set_err("lbm_surrogate_train: bad training configuration");
    return LBM_EINVAL;
  }
  if (!all_finite(feat, (size_t)n * sg::kFeat) || !all_finite(target, (size_t)n * sg::kOut)) {
    set_err("lbm_surrogate_train: data must be finite");
    return LBM_ENONFINITE;
  }
  const int Mb = s->members;
  if (order) {
    for (long long i = 0; i < (long long)cfg->epochs * Mb * n; ++i)
      if (order[i] < 0 || order[i] >= n) {
        set_err("lbm_surrogate_train: order[%lld] = %d is not a sample index", i, order[i]);
        return LBM_EINVAL;
      }
  }
  // statistics from the data (FP64 on the device), then standardised copies
  double *raw = nullptr;
  SGTRY(dalloc(&raw, (size_t)n * sg::kFeat));
  SGCHK(hipMemcpyAsync(raw, feat, sizeof(double) * n * sg::kFeat, hipMemcpyHostToDevice,
                       s->stream));
  SGCHK(sg::launch_col_stats(raw, n, sg::kFeat, s->xmu(), s->xsd(), s->stream));
  SGCHK(hipStreamSynchronize(s->stream));
  dfree(raw);
  SGTRY(dalloc(&raw, (size_t)n * sg::kOut));
  SGCHK(hipMemcpyAsync(raw, target, sizeof(double) * n * sg::kOut, hipMemcpyHostToDevice,
                       s->stream));
  SGCHK(sg::launch_col_stats(raw, n, sg::kOut, s->tmu(), s->tsd(), s->stream));
  SGCHK(hipStreamSynchronize(s->stream));
  dfree(raw);
  s->has_stats = true;
  float *xs_d = nullptr, *ts_d = nullptr;
  int *idx_d = nullptr;
  SGTRY(upload_std(s, feat, n, sg::kFeat, s->xmu(), s->xsd(), &xs_d));
  int rc = upload_std(s, target, n, sg::kOut, s->tmu(), s->tsd(), &ts_d);
  if (rc == LBM_OK) rc = dalloc(&idx_d, (size_t)Mb * n);
  const int bsz_max = std::min(cfg->batch, n);
  if (rc == LBM_OK) rc = s->ensure(bsz_max);
  // sample order: given, or each member's bootstrap resample (or the full
  // set) shuffled per epoch by Fisher-Yates, both driven by SplitMix64
  std::vector<int> base((size_t)Mb * n), ord((size_t)Mb * n);
  if (!order)
    for (int z = 0; z < Mb; ++z)
      for (int j = 0; j < n; ++j)
        base[(size_t)z * n + j] =
            cfg->bootstrap ? (int)(splitmix64(cfg->seed ^ (0x5851F42D4C957F2Dull * (z + 1)), j) %
                                   (uint64_t)n)
                           : j;
  const int per_epoch = (n + cfg->batch - 1) / cfg->batch;
  const long long total = (long long)cfg->epochs * per_epoch;
  std::vector<double> lsum(Mb), lstep(Mb);
  for (int e = 0; e < cfg->epochs && rc == LBM_OK; ++e) {
    if (order) {
      std::memcpy(ord.data(), order + (size_t)e * Mb * n, sizeof(int) * Mb * n);
    } else {
      ord = base;
      for (int z = 0; z < Mb; ++z) {
        int *o = ord.data() + (size_t)z * n;
        const uint64_t sd = splitmix64(cfg->seed, (uint64_t)e * 65536u + (uint64_t)z);
        for (int j = n - 1; j > 0; --j) std::swap(o[j], o[splitmix64(sd, j) % (uint64_t)(j + 1)]);
      }
    }
    hipError_t he = hipMemcpyAsync(idx_d, ord.data(), sizeof(int) * Mb * n,
                                   hipMemcpyHostToDevice, s->stream);
    if (he != hipSuccess) {
      set_err("order upload failed: %s", hipGetErrorString(he));
      rc = LBM_EHIP;
      break;
    }
    std::fill(lsum.begin(), lsum.end(), 0.0);
    for (int st = 0; st < per_epoch && rc == LBM_OK; ++st) {
      const int start = st * cfg->batch, cnt = std::min(cfg->batch, n - start);
      he = sg::launch_gather(xs_d, ts_d, idx_d + start, n, Mb, cnt, s->cap, s->act[0], s->t,
                             s->stream);
      if (he != hipSuccess) {
        set_err("gather failed: %s", hipGetErrorString(he));
        rc = LBM_EHIP;
        break;
      }
      rc = s->forward(cnt, (long long)s->cap * sg::kFeat);
      if (rc == LBM_OK) rc = s->backward(cnt);
      if (rc != LBM_OK) break;
      const long long step = (long long)e * per_epoch + st;
      const double cosw = 0.5 * (1.0 + std::cos(M_PI * (double)step / (double)std::max(total, 1LL)));
      const double lr = cfg->lr * (cfg->lr_min_frac + (1.0 - cfg->lr_min_frac) * cosw);
      s->adam_t += 1;
      const double bc1 = 1.0 - std::pow(cfg->beta1, (double)s->adam_t);
      const double bc2 = 1.0 - std::pow(cfg->beta2, (double)s->adam_t);
      he = sg::launch_adam(s->w, s->g, s->m, s->v, s->wb, (long long)Mb * P, (float)lr,
                           (float)cfg->beta1, (float)cfg->beta2, (float)cfg->eps, (float)bc1,
                           (float)bc2, s->stream);
      if (he == hipSuccess && loss_hist)
        he = hipMemcpyAsync(lstep.data(), s->loss_d, sizeof(double) * Mb, hipMemcpyDeviceToHost,
                            s->stream);
      if (he == hipSuccess && loss_hist) he = hipStreamSynchronize(s->stream);
      if (he != hipSuccess) {
        set_err("training step failed: %s", hipGetErrorString(he));
        rc = LBM_EHIP;
        break;
      }
      if (loss_hist)
        for (int z = 0; z < Mb; ++z) lsum[z] += lstep[z];
    }
    if (rc == LBM_OK && loss_hist) {
      double a = 0;
      for (int z = 0; z < Mb; ++z) a += lsum[z] / per_epoch;
      loss_hist[e] = a / Mb;
    }
  }
  if (rc == LBM_OK && hipStreamSynchronize(s->stream) != hipSuccess) {
    set_err("training did not complete");
    rc = LBM_EHIP;
  }
  dfree(xs_d);
  dfree(ts_d);
  dfree(idx_d);
  return rc;
}

namespace {

// predictions for n raw descriptor rows already on the device
int predict_device(lbm_surrogate_t s, const double *feat_d, int n, double *mean_d, double *std_d) {
  float *xs_d = nullptr;
  SGTRY(dalloc(&xs_d, (size_t)n * sg::kFeat));
  hipError_t e = sg::launch_standardise(feat_d, n, sg::kFeat, s->xmu(), s->xsd(), xs_d, s->stream);
  if (e != hipSuccess) {
    dfree(xs_d);
    set_err("standardise failed: %s", hipGetErrorString(e));
    return LBM_EHIP;
  }
  int rc = forward_chunks(s, xs_d, n, [&](int start, int cnt) -> int {
    SGCHK(sg::launch_ensemble(s->y, s->members, cnt, s->cap, s->tmu(), s->tsd(),
                              mean_d + (size_t)start * sg::kOut, std_d + (size_t)start * sg::kOut,
                              s->stream));
    return LBM_OK;
  });
  if (rc == LBM_OK && hipStreamSynchronize(s->stream) != hipSuccess) {
    set_err("prediction did not complete");
    rc = LBM_EHIP;
  }
  dfree(xs_d);
  return rc;
}

}  // namespace

int lbm_surrogate_predict(lbm_surrogate_t s, int n, const double *feat, double *mean,
                          double *std) {
  SGTRY(check_model(s));
  if (n < 0 || (n > 0 && (!feat || !mean || !std))) {
    set_err("lbm_surrogate_predict: bad arguments");
    return LBM_EINVAL;
  }
  if (!s->has_stats) {
    set_err("lbm_surrogate_predict: the model has no standardisation statistics");
    return LBM_ESTATE;
  }
  if (n == 0) return LBM_OK;
  if (!all_finite(feat, (size_t)n * sg::kFeat)) {
    set_err("lbm_surrogate_predict: features must be finite");
    return LBM_ENONFINITE;
  }
  double *f_d = nullptr, *mean_d = nullptr, *std_d = nullptr;
  SGTRY(dalloc(&f_d, (size_t)n * sg::kFeat));
  int rc = dalloc(&mean_d, (size_t)n * sg::kOut);
  if (rc == LBM_OK) rc = dalloc(&std_d, (size_t)n * sg::kOut);
  if (rc == LBM_OK && hipMemcpyAsync(f_d, feat, sizeof(double) * n * sg::kFeat,
                                     hipMemcpyHostToDevice, s->stream) != hipSuccess) {
    set_err("feature upload failed");
    rc = LBM_EHIP;
  }
  if (rc == LBM_OK) rc = predict_device(s, f_d, n, mean_d, std_d);
  if (rc == LBM_OK) {
    hipError_t e = hipMemcpyAsync(mean, mean_d, sizeof(double) * n * sg::kOut,
                                  hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(std, std_d, sizeof(double) * n * sg::kOut, hipMemcpyDeviceToHost,
                         s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
      set_err("prediction download failed: %s", hipGetErrorString(e));
      rc = LBM_EHIP;
    }
  }
  dfree(f_d);
  dfree(mean_d);
  dfree(std_d);
  return rc;
}

int lbm_surrogate_pce(lbm_surrogate_t s, int n, const lbm_params *p, const double *pc, int n_pc,
                      const lbm_conv *c, double threshold, int run_fallback, double *pce,
                      double *curve, double *pce_std, int *used_fallback, lbm_sg_info *info) {
  SGTRY(check_model(s));
  if (n < 1 || !p || !pce || !curve || !pce_std || !used_fallback || !(threshold >= 0)) {
    set_err("lbm_surrogate_pce: bad arguments");
    return LBM_EINVAL;
  }
  if (run_fallback && (!pc || !c || n_pc != LBM_SG_NCURVE)) {
    set_err("lbm_surrogate_pce: the LBM fallback needs pc [n][%d] and a convergence setting",
            LBM_SG_NCURVE);
    return LBM_EINVAL;
  }
  if (!s->has_stats) {
    set_err("lbm_surrogate_pce: the model has no standardisation statistics");
    return LBM_ESTATE;
  }
  std::vector<double> geo;
  SGTRY(params_geometry(n, p, geo));
  double *geo_d = nullptr, *feat_d = nullptr, *mean_d = nullptr, *std_d = nullptr;
  SGTRY(dalloc(&geo_d, geo.size()));
  int rc = dalloc(&feat_d, (size_t)n * sg::kFeat);
  if (rc == LBM_OK) rc = dalloc(&mean_d, (size_t)n * sg::kOut);
  if (rc == LBM_OK) rc = dalloc(&std_d, (size_t)n * sg::kOut);
  float t_desc = 0.f, t_pred = 0.f;
  if (rc == LBM_OK) {
    hipError_t e = hipMemcpyAsync(geo_d, geo.data(), sizeof(double) * geo.size(),
                                  hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ev[0], s->stream);
    if (e == hipSuccess) e = sg::launch_describe(geo_d, n, feat_d, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ev[1], s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t_desc, s->ev[0], s->ev[1]);
    if (e != hipSuccess) {
      set_err("descriptor failed: %s", hipGetErrorString(e));
      rc = LBM_EHIP;
    }
  }
  if (rc == LBM_OK) {
    (void)hipEventRecord(s->ev[0], s->stream);
    rc = predict_device(s, feat_d, n, mean_d, std_d);
    (void)hipEventRecord(s->ev[1], s->stream);
    (void)hipEventSynchronize(s->ev[1]);
    (void)hipEventElapsedTime(&t_pred, s->ev[0], s->ev[1]);
  }
  std::vector<double> mean((size_t)n * sg::kOut), sd((size_t)n * sg::kOut);
  if (rc == LBM_OK) {
    hipError_t e = hipMemcpyAsync(mean.data(), mean_d, sizeof(double) * mean.size(),
                                  hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(sd.data(), std_d, sizeof(double) * sd.size(), hipMemcpyDeviceToHost,
                         s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
      set_err("prediction download failed: %s", hipGetErrorString(e));
      rc = LBM_EHIP;
    }
  }
  dfree(geo_d);
  dfree(feat_d);
  dfree(mean_d);
  dfree(std_d);
  if (rc != LBM_OK) return rc;

  std::vector<int> fb;
  for (int t = 0; t < n; ++t) {
    const double r_msp = msp_radius(geo.data() + (size_t)t * 19);
    const double m0 = mean[(size_t)t * sg::kOut], s0 = sd[(size_t)t * sg::kOut];
    pce[t] = r_msp > 0 ? m0 / r_msp : NAN;
    pce_std[t] = r_msp > 0 ? s0 / r_msp : NAN;
    for (int j = 0; j < LBM_SG_NCURVE; ++j)
      curve[(size_t)t * LBM_SG_NCURVE + j] = mean[(size_t)t * sg::kOut + 1 + j];
    // (no MS-P radius: no network answer, the LBM decides)
    const bool disagree = !(s0 <= threshold * std::fabs(m0)) || !(r_msp > 0);
    used_fallback[t] = 0;
    if (disagree && run_fallback) fb.push_back(t);
  }
  int status = LBM_OK;
  lbm_batch_info bi{};
  double lbm_ms = 0.0;
  if (!fb.empty()) {
    const int nf = (int)fb.size();
    std::vector<lbm_params> sub((size_t)nf);
    std::vector<double> pcs((size_t)nf * n_pc), S((size_t)nf * n_pc);
    std::vector<long long> steps((size_t)nf * n_pc);
    std::vector<int> stat((size_t)nf * n_pc);
    std::vector<lbm_drain_result> res((size_t)nf);
    for (int i = 0; i < nf; ++i) {
      sub[i] = p[fb[i]];
      std::memcpy(pcs.data() + (size_t)i * n_pc, pc + (size_t)fb[i] * n_pc, sizeof(double) * n_pc);
      res[i] = lbm_drain_result{};
      res[i].S = S.data() + (size_t)i * n_pc;
      res[i].steps = steps.data() + (size_t)i * n_pc;
      res[i].status = stat.data() + (size_t)i * n_pc;
    }
    status = lbm_drain_batch(nf, sub.data(), pcs.data(), n_pc, c, res.data(), &bi);
    if (status < 0) return status;
    lbm_ms = bi.wall_ms;
    for (int i = 0; i < nf; ++i) {
      const int t = fb[i];
      // 2: the LBM answer failed (non-finite state), so there is none
      used_fallback[t] = res[i].failed ? 2 : 1;
      pce[t] = res[i].failed ? NAN : res[i].pce;
      pce_std[t] = res[i].failed ? NAN : 0.0;
      for (int j = 0; j < LBM_SG_NCURVE; ++j) curve[(size_t)t * LBM_SG_NCURVE + j] = S[(size_t)i * n_pc + j];
    }
  }
  if (info) {
    info->n_fallback = (int)fb.size();
    info->describe_ms = t_desc;
    info->predict_ms = t_pred;
    info->lbm_ms = lbm_ms;
    info->lbm = bi;
  }
  return status;
}

}  // extern "C"
