// sc_internal.h -- device-side data structures and kernel launchers of the
// Shan-Chen throat library (internal; the public interface is lbm_abi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace sc {

// node classes, stored in bits 24..25 of the per-node mask word; bits 0..18
// flag the directions k whose pull source x - e_k is solid or beyond a wall
enum : uint32_t { kFluid = 0, kSolid = 1, kResIn = 2, kResOut = 3 };
constexpr int kTypeShift = 24;

// one subdomain's storage: shifted FP32 populations g = f - w_k rho_ref in
// structure-of-arrays order [component][direction][node]
struct Dom {
  const float *src;      // post-collision state of the previous step
  float *dst;            // post-collision state written by this step
  const uint32_t *mask;  // [N] link bits + node class
  size_t N;              // nodes = nx * ny * nz (plane stride)
  int nx, ny, nz;
  int per;               // bit 0/1/2: x/y/z periodic
};

// physical parameters in the precision the step computes in
struct Phys {
  float tau[2], itau[2];
  float G, Gads[2];
  float rho_ref;         // shift of the stored populations
  float rres[2][2];      // bath densities [in/out][component]
  float gres[2][2];      // rres - rho_ref
};

// launch shape of the fused step
struct Sched {
  int tx, ty, lz;
};

// one subdomain as the fused step sees it: both population buffers, the
// mask, the size, the tile grid of the launch schedule and the parameters
// (a launch covers the tiles of one or many of these)
struct Throat {
  float *g[2];           // A/B buffers; the state is in g[parity]
  const uint32_t *mask;
  uint32_t N;
  int nx, ny, nz, per;
  int ntx, nty, lz;      // tile grid: tiles of TX x TY nodes and lz planes
  int active;            // 0: the launch skips this subdomain
  Phys P;
};

// one tile of work: subdomain index and packed tile coordinate
// tix + ntx * (tiy + nty * tiz)
struct TileRef {
  int throat;
  int tile;
};

// kernel launchers (all asynchronous on `st`)
hipError_t launch_voxelize(const double *spheres, int n_spheres, int prism, const int *prism_ids,
                           int nx, int ny, int nz, int bc_z_reservoir, uint8_t *types,
                           hipStream_t st);
hipError_t launch_links(const uint8_t *types, int nx, int ny, int nz, int per, uint32_t *mask,
                        hipStream_t st);
hipError_t launch_init(const Dom &d, const Phys &P, const double *rho_init, double rho_major,
                       double rho_minor, int z_front, const double *rres_d, float *g,
                       hipStream_t st);
// one time step of every active subdomain in `throats` over the listed tiles
// (device arrays); tx, ty is the tile shape the lists were built for
hipError_t launch_step(const Throat *throats, const TileRef *tiles, int ntiles, int tx, int ty,
                       int parity, hipStream_t st);
// host: append the tiles of subdomain `throat` that hold at least one
// non-solid node (solid-only tiles need no update)
void list_tiles(const uint8_t *types, int nx, int ny, int nz, int tx, int ty, int lz, int throat,
                std::vector<TileRef> &out);
hipError_t launch_export(const Dom &d, const Phys &P, const double *rres_d, double *f,
                         hipStream_t st);
hipError_t launch_density(const Dom &d, const Phys &P, const double *rres_d, double *rho,
                          hipStream_t st);
// FP64 reduction: out[0..1] masses, out[2] sum of the saturation term,
// out[3..4] densities at the probe node (if probe >= 0)
hipError_t launch_reduce(const Dom &d, const Phys &P, double phib, long long probe,
                         double *partials, int n_partials, double *out, hipStream_t st);
int reduce_blocks(size_t N);
// plain copy of n_floats (a multiple of 4) floats, 16-byte aligned buffers
hipError_t launch_copy(const float *a, float *b, size_t n_floats, hipStream_t st);

bool schedule_valid(const Sched &s);

}  // namespace sc
