// lbm_handle.h -- the subdomain handle behind lbm_throat_t and the host
// helpers shared by the single-subdomain and the batched entry points
// (internal; the public interface is lbm_abi.h).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "lbm_abi.h"
#include "sc_internal.h"

// host-side drainage ramp of one subdomain (Sec. 2.2.2), advanced in chunks
// of check_every steps so that a caller can stop it, save it and resume it
struct HostRamp {
  enum : int { kIdle = 0, kRamp = 1, kBisect = 2, kDone = 3 };
  int phase = kIdle;
  std::vector<double> pc;
  lbm_conv c{};
  int point = 0;                // ramp point being run (kRamp) or bisected (kBisect)
  // the run in progress: steps so far and the saturation of the last check
  long long run_steps = 0;
  double S_old = 0.0;
  // bracket of the entry pressure and the states kept for the bisection
  double stable_pc = 0.0, lo = 0.0, hi = 0.0, mid = 0.0, main_rho_in = 0.0;
  int inv_at = -1, n_bisect = 0, runs = 0, warn = 0, failed = 0;
  long long total = 0;
  std::vector<double> S;
  std::vector<long long> steps;
  std::vector<int> status;
};

struct lbm_throat {
  int nx = 0, ny = 0, nz = 0, per = 0, bc[3] = {0, 0, 0};
  size_t N = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *g[2] = {nullptr, nullptr};  // A/B population buffers
  int cur = 0;                       // g[cur] holds the current state
  float *save[2] = {nullptr, nullptr};  // checkpoints used by the ramp
  uint32_t *mask = nullptr;
  uint2 *list_d = nullptr;           // non-solid nodes, storage order, with mask (node-list path)
  uint32_t nlist = 0;
  float2 *rho_d = nullptr;           // densities of the current step (node-list path)
  uint8_t *types_d = nullptr;
  double *rres_d = nullptr;          // [in/out][component]
  // chunked FP64 reduction: node chunks, per-chunk partials, sums + probe
  sc::Chunk *chunks_d = nullptr;
  int nchunks = 0;
  sc::RedInfo *redinfo_d = nullptr;
  int *chunk_first_d = nullptr;      // [1] = 0
  int *chunk_count_d = nullptr;      // [1] = nchunks
  double *partials = nullptr;        // [nchunks][3]
  double *red_d = nullptr;           // [5]: masses, saturation sum, probe densities
  double *red_h = nullptr;           // pinned [5]
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<uint8_t> types;
  std::vector<uint8_t> bricks;       // brick liveness map (sc::brick_map)
  size_t n_nonsolid = 0;
  long long n_fluid = 0;
  long long probe = -1;
  double tau[2], G, Gads[2], rho_major, rho_minor, rho_in, rho_out;
  double phib = 1.0;
  sc::Phys P{};
  sc::Sched sched{64, 4, 16};
  long long steps_done = 0;
  // device descriptor and tile list of the fused step
  sc::Throat desc{};
  sc::Throat *desc_d = nullptr;
  sc::TileRef *tiles_d = nullptr;
  int ntiles = 0;
  size_t tiles_cap = 0;
  int *zper_d = nullptr;             // {0} on a z-periodic subdomain (ghost planes)
  int n_zper = 0;
  // event-timed step launches inside the drainage ramp
  hipEvent_t tev[2] = {nullptr, nullptr};
  bool timing = false;
  double timed_ms = 0.0;
  long long timed_launches = 0;
  HostRamp ramp;
};


namespace lbmh {

void set_err(const char *fmt, ...);
// refresh the device descriptor / rebuild the tile list of the schedule
int sync_desc(lbm_throat *h);
int rebuild_tiles(lbm_throat *h);
int set_rho_in(lbm_throat *h, double r);
int copy_state(lbm_throat *h, float *dst, const float *src);
// device memory of one subdomain (with or without the two ramp checkpoints)
// and the refusal of a call whose need exceeds the memory budget
size_t subdomain_bytes(int nx, int ny, int nz, bool checkpoints);
int check_budget(size_t need, const char *what);

}  // namespace lbmh
