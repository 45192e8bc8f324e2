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
// bits 1..18 of a mask word: link k is cut (x - e_k solid or beyond a wall)
constexpr uint32_t kLinkBits = 0x7FFFEu;

// Population storage of one buffer: shifted FP32 populations g = f - w_k
// rho_ref, q = 19 c + k for component c and direction k.  Each z-plane is cut
// into bricks of 8 x 4 nodes (x, y; the plane padded to multiples of 8 and 4)
// and a brick holds its 38 populations one after another, each a run of 32
// floats (one 128-byte line) in (y mod 4, x mod 8) order: element (q, x, y, z)
// is at (z + 1) Pp + ((y / 4) (nxp / 8) + x / 8) 38 * 32 + 32 q + 8 (y mod 4)
// + x mod 8, Pp = 38 nxp nyp.  A line then holds a compact 8 x 4 patch of one
// population, so the sparse, irregular fluid of a throat box wastes fewer
// fetched bytes than with runs along x (1.55 against 2.44 fetched per useful
// byte on a 96^3 four-sphere throat), and the 38 values of four rows of nodes
// still share one 608 nxp-byte range.  Planes z = -1 and z = nz are ghost
// copies of planes nz - 1 and 0 on z-periodic subdomains (unused otherwise),
// so that the pulls of a node on plane z read planes z - 1 .. z + 1 only: one
// base address and 32-bit offsets.
constexpr int kQ = 38;
constexpr int kBX = 8, kBY = 4, kBN = kBX * kBY;  // brick of one 128-byte line
#ifndef SC_BRICK_OX
#define SC_BRICK_OX 0
#endif
#ifndef SC_BRICK_OY
#define SC_BRICK_OY 0
#endif
constexpr int kOX = SC_BRICK_OX, kOY = SC_BRICK_OY;
__host__ __device__ inline int pad_x(int nx) { return (nx + kOX + kBX - 1) / kBX * kBX; }
__host__ __device__ inline int pad_y(int ny) { return (ny + kOY + kBY - 1) / kBY * kBY; }
__host__ __device__ inline size_t pop_plane(int nx, int ny) {
  return (size_t)kQ * pad_x(nx) * pad_y(ny);
}
__host__ __device__ inline size_t pop_elems(int nx, int ny, int nz) {
  return pop_plane(nx, ny) * (size_t)(nz + 2);
}
// offset of population 0 of node (x, y) within its plane (0 <= x < nx,
// 0 <= y < ny); population q is 32 q further
__host__ __device__ inline uint32_t brick_x(int x) {
  return (uint32_t)((x + kOX) / kBX) * (uint32_t)(kQ * kBN) + (uint32_t)((x + kOX) % kBX);
}
__host__ __device__ inline uint32_t brick_y(int y, int nx) {
  return (uint32_t)((y + kOY) / kBY) * (uint32_t)(pad_x(nx) / kBX) * (uint32_t)(kQ * kBN) +
         (uint32_t)((y + kOY) % kBY) * (uint32_t)kBX;
}
// largest padded nx * ny whose three-plane pull offsets fit 32 bits of bytes
constexpr long long kMaxPlaneNodes = (1LL << 32) / (3LL * kQ * 4) - 1;

// one subdomain as the per-node kernels see it
struct Dom {
  const float *src;      // post-collision state of the previous step
  float *dst;            // post-collision state written by this step
  const uint32_t *mask;  // [N] link bits + node class
  size_t N;              // nodes = nx * ny * nz
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

// launch shape of the step: tiles of tx x ty columns marching lz planes in
// one fused pass, or (tx = kListTx) the node-list path of two passes over
// the non-solid nodes only (densities, then the fused pull-collide-store)
struct Sched {
  int tx, ty, lz;
};
constexpr int kListTx = -1;

// tile shapes (tx, ty) the fused step is built for; lz is free (>= 1).  The
// narrow shapes fit thin prism subdomains with fewer solid columns per tile.
constexpr int kNumShapes = 6;
constexpr int kShapes[kNumShapes][2] = {{32, 4}, {32, 8}, {64, 4}, {16, 4}, {16, 8}, {8, 8}};

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
  const uint2 *list;     // node-list path: non-solid nodes in storage order (index, mask word)
  uint32_t nlist;
  float2 *rho;           // node-list path: densities of the current step [N]
  Phys P;
};

// node-list path: one workgroup of kListBlock threads per kListNodes
// consecutive entries of a subdomain's node list (TileRef::tile = chunk), a
// pair of lanes per node (one per component)
constexpr int kListBlock = 256;
constexpr int kListNodes = kListBlock / 2;

// one tile of work: subdomain index and packed tile coordinate
// tix + ntx * (tiy + nty * tiz)
struct TileRef {
  int throat;
  int tile;
};

// spheres binned into cubic cells of kVoxCell nodes (CSR lists, device)
constexpr int kVoxCell = 16;
struct VoxBins {
  const int *start;  // [ncells + 1]
  const int *ids;    // sphere indices, increasing within a cell
  int ncx, ncy, ncz;
};
// host side of the binning: every sphere goes to each cell that its bounding
// box, widened by one node, meets
void bin_spheres(const double *sph, int ns, int nx, int ny, int nz, std::vector<int> &start,
                 std::vector<int> &ids, int &ncx, int &ncy, int &ncz);

// kernel launchers (all asynchronous on `st`)
hipError_t launch_voxelize(const double *spheres, const VoxBins &bins, int prism,
                           const int *prism_ids, int nx, int ny, int nz, int bc_z_reservoir,
                           uint8_t *types, hipStream_t st);
hipError_t launch_links(const uint8_t *types, int nx, int ny, int nz, int per, uint32_t *mask,
                        hipStream_t st);
// node-list entries: out[i] = (ids[i], mask[ids[i]]) for i < n
hipError_t launch_list_entries(const uint32_t *ids, const uint32_t *mask, uint32_t n, uint2 *out,
                               hipStream_t st);
hipError_t launch_init(const Dom &d, const Phys &P, const double *rho_init, double rho_major,
                       double rho_minor, int z_front, const double *rres_d, float *g,
                       hipStream_t st);
// one time step of every active subdomain in `throats` over the listed tiles
// (device arrays); tx, ty is the tile shape the lists were built for.
// zper_ids (device, n_zper entries): the z-periodic subdomains, whose ghost
// planes are refreshed after the step.
hipError_t launch_step(const Throat *throats, const TileRef *tiles, int ntiles, int tx, int ty,
                       int parity, hipStream_t st, const int *zper_ids, int n_zper);
// host: per plane, which 8 x 4 bricks hold a non-solid node ([nz][nyp / 4]
// [nxp / 8] bytes), and the number of non-solid nodes; computed once per
// subdomain from its node classes
void brick_map(const uint8_t *types, int nx, int ny, int nz, std::vector<uint8_t> &live,
               size_t &nonsolid);
// host: append the tiles of subdomain `throat` that hold at least one
// non-solid node (solid-only tiles need no update), from its brick map; every
// tile shape is a whole number of bricks
void list_tiles(const uint8_t *live, size_t nonsolid, int nx, int ny, int nz, int tx, int ty,
                int lz, int throat, std::vector<TileRef> &out);
hipError_t launch_export(const Dom &d, const Phys &P, const double *rres_d, double *f,
                         hipStream_t st);
hipError_t launch_density(const Dom &d, const Phys &P, const double *rres_d, double *rho,
                          hipStream_t st);
// fixed device staging array of the allocation-free density read-back:
// kScratchDoubles doubles (32 MiB), enough for 2 densities of 2^21 nodes (a
// 128^3 box).  scratch_address gives the device address of the current
// device's copy (looked up once per device, then cached).
constexpr size_t kScratchNodes = (size_t)1 << 21;
constexpr size_t kScratchDoubles = 2 * kScratchNodes;
hipError_t scratch_address(double **out);
// chunked FP64 reduction over subdomains: each reduction chunk is a range of
// kRedEntries entries of one subdomain's node list; per chunk the partial
// sums of rho_w, rho_nw and the saturation term over its fluid nodes, then
// per subdomain the sum of its chunks in order.  Copy chunks (the batch's
// checkpoint copies) split each subdomain's buffer by node ranges of
// kChunkNodes instead, so that a copy gets blocks in proportion to its size.
struct Chunk {
  int throat;
  uint32_t start, count;
};
struct RedInfo {
  long long probe;  // probe node or -1
  double phib;      // bulk order parameter of the saturation map
};
constexpr uint32_t kChunkNodes = 4096;
constexpr uint32_t kRedEntries = 1024;
void list_chunks(int throat, uint32_t N, std::vector<Chunk> &out);
void list_red_chunks(int throat, uint32_t nlist, std::vector<Chunk> &out);
// partials[c][3]; probe_out[t][2] = densities at subdomain t's probe node
hipError_t launch_reduce_chunks(const Throat *th, const Chunk *chunks, int nchunks,
                                const RedInfo *info, int parity, double *partials,
                                double *probe_out, hipStream_t st);
// sums[t][3] = sum over chunks first[t] .. first[t]+count[t]-1, in order
hipError_t launch_reduce_throats(const int *first, const int *count, int n, const double *partials,
                                 double *sums, hipStream_t st);
// plain copy of n_floats (a multiple of 4) floats, 16-byte aligned buffers
hipError_t launch_copy(const float *a, float *b, size_t n_floats, hipStream_t st);

bool schedule_valid(const Sched &s);

// ---- device-side drainage ramp of a batch of subdomains -------------------
enum : int { kPhaseRamp = 0, kPhaseBisect = 1, kPhaseDone = 2 };
// copy requests executed after each ramp decision, saves before restores
enum : int { kSaveStable = 1, kSaveMain = 2, kRestoreStable = 4, kRestoreMain = 8 };

// bisection runs of one drain at most: a throat already invaded at the first
// ramp point has 0 as its lower bracket, where halving alone need not reach
// the relative width; the drain then ends with its bracket and a warning
constexpr int kMaxBisect = 40;

struct RampCfg {
  double tol;        // |S(t) - S(t - every)| < tol ends a ramp point
  double rel;        // bisection stops at (hi - lo) / hi <= rel
  long long cap;     // steps per ramp point or bisection run
  int every;         // steps between checks (even)
  int n_pc;
};

struct RampDev {
  double rho_out, dpc_drho, rho_ref;   // rho_in = rho_out + pc / dpc_drho
  double S_old, S_stable, S_main, lo, hi, mid, stable_pc, rho_in_main;
  long long steps_pt, total_steps;
  unsigned int n_fluid;
  int phase, point, invaded_at, n_bisect, req, warn, failed;
};

struct Ckpt {
  float *stable, *main;
};

// first decision: record the initial saturation, save it as the stable
// state, set the first inlet density
hipError_t launch_ramp_begin(Throat *th, RampDev *rd, const double *pc, const RampCfg &cfg,
                             const double *sums, int n, hipStream_t st);
// one decision per subdomain after `every` steps; n_active_out[0] = number of
// subdomains still running
hipError_t launch_ramp_advance(Throat *th, RampDev *rd, const double *pc, const RampCfg &cfg,
                               const double *sums, const double *probe, double *S_out,
                               long long *steps_out, int *status_out, int n, int *n_active_out,
                               hipStream_t st);
// perform the copy requests of every subdomain (over the reduction chunks)
hipError_t launch_copy_requests(const Throat *th, const RampDev *rd, const Ckpt *ck,
                                const Chunk *chunks, int nchunks, int parity, hipStream_t st);

}  // namespace sc
