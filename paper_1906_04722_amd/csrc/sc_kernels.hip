// sc_kernels.hip -- gfx950 kernels of the two-component Shan-Chen D3Q19
// update (Montella et al., Sec. 2.1, Eq. 1-5) on one pore-throat subdomain.
//
// Storage: shifted FP32 populations g = f - w_k rho_ref in bricks of 8 x 4
// nodes per z-plane, each population of a brick one 128-byte line, so that
// the 64 lanes of a wavefront read and write two whole lines per population
// (layout and ghost planes in sc_internal.h).  The update is a
// pull scheme: buffer `src` holds the post-collision state of step t-1 at
// each node's own position; pulling g_k from x - e_k gives the pre-collision
// state f(x, t) of Eq. 1.  One kernel does the whole step: pull + half-way
// bounce-back, moments (Eq. 2-3), the cohesion force (Eq. 4) from an LDS ring
// of density planes, the adhesion force from the node's link bits, the
// velocity shift, BGK relaxation toward the component equilibria (Eq. 1) and
// the store of the post-collision state.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "geom.h"
#include "sc_internal.h"

// Multiply-adds are fused only where one source expression reads a * b + c,
// never across statements, so every kernel that shares the arithmetic below
// (the tiled step, the node-list step, the export) rounds it identically.
#pragma clang fp contract(on)

namespace sc {

// ---- D3Q19: rest; +x,-x,+y,-y,+z,-z; twelve edges, opposite pairs adjacent
__host__ __device__ constexpr int ex(int k) {
  constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[k];
}
__host__ __device__ constexpr int ey(int k) {
  constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[k];
}
__host__ __device__ constexpr int ez(int k) {
  constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[k];
}
__host__ __device__ constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }
__host__ __device__ constexpr float wf(int k) {
  return k == 0 ? 1.0f / 3.0f : (k <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr double wd(int k) {
  return k == 0 ? 1.0 / 3.0 : (k <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---- node addressing ------------------------------------------------------

// Map (X, Y, Z), which may lie one node beyond the box, to a node index:
// wrapped on periodic axes, -1 beyond a wall.  Coordinates further out (the
// unused halo slots of a ragged tile) also give -1.
__device__ __forceinline__ long long node_of(const Dom &d, int X, int Y, int Z) {
  if (X < -1 || X > d.nx || Y < -1 || Y > d.ny || Z < -1 || Z > d.nz) return -1;
  if (X < 0 || X >= d.nx) {
    if (!(d.per & 1)) return -1;
    X = X < 0 ? X + d.nx : X - d.nx;
  }
  if (Y < 0 || Y >= d.ny) {
    if (!(d.per & 2)) return -1;
    Y = Y < 0 ? Y + d.ny : Y - d.ny;
  }
  if (Z < 0 || Z >= d.nz) {
    if (!(d.per & 4)) return -1;
    Z = Z < 0 ? Z + d.nz : Z - d.nz;
  }
  return (long long)X + (long long)d.nx * ((long long)Y + (long long)d.ny * Z);
}

__device__ __forceinline__ int wrap(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// Pull the pre-collision populations f(x,t) - w_k rho_ref of the fluid node
// at (X, Y, Z) with link bits m: g_k from x - e_k, or the reflected g_opp(k)
// at x itself when the link to x - e_k is cut by a solid node or a wall
// (half-way bounce-back).  Addresses are the start of plane Z - 1 (uniform
// across a tile) plus a 32-bit byte offset per lane.  In the brick storage
// the offset of a node is the sum of an x part and a y part (brick_x,
// brick_y); with P the elements of a plane, population q of the node itself
// is at P + y(Y) + x(X) + 32 q, of the source node at (1 - ez) P + y(Ys) +
// x(Xs) + 32 q.  The second component's populations follow 19 * 32 later.
// Xs and Ys are taken modulo nx and ny: across a periodic face that is the
// wrapped neighbour, across a wall the link is cut and the offset unused.
// global-memory views of the population buffers: loads and stores then take
// a uniform 64-bit base and a 32-bit per-lane offset
typedef const __attribute__((address_space(1))) char gcchar;
typedef __attribute__((address_space(1))) char gchar;

template <int K>
__device__ __forceinline__ void pull_dir(gcchar *b0, gcchar *b1, uint32_t m, uint32_t own,
                                         uint32_t s, float (&v)[2][19]) {
  constexpr int o = opp(K);
  const bool cut = (m >> K) & 1u;
  const uint32_t off = cut ? own + (uint32_t)(o * kBN) : s + (uint32_t)(K * kBN);
  v[0][K] = *(const __attribute__((address_space(1))) float *)(b0 + (size_t)(off * 4u));
  v[1][K] = *(const __attribute__((address_space(1))) float *)(b1 + (size_t)(off * 4u));
}

// source offset of direction K: planes, then the y and x parts of x - e_k
// (index 0: coordinate - 1, 1: itself, 2: + 1)
template <int K>
__device__ __forceinline__ uint32_t src_index(uint32_t P, const uint32_t (&py)[3],
                                              const uint32_t (&px)[3]) {
  return (uint32_t)(1 - ez(K)) * P + py[1 - ey(K)] + px[1 - ex(K)];
}

template <int K>
__device__ __forceinline__ void pull_rec(gcchar *b0, gcchar *b1, uint32_t m, uint32_t own,
                                         uint32_t P, const uint32_t (&py)[3],
                                         const uint32_t (&px)[3], float (&v)[2][19]) {
  pull_dir<K>(b0, b1, m, own, src_index<K>(P, py, px), v);
  if constexpr (K + 1 < 19) pull_rec<K + 1>(b0, b1, m, own, P, py, px, v);
}

__device__ __forceinline__ void pull(const Dom &d, uint32_t m, int X, int Y, int Z,
                                     float (&v)[2][19]) {
  const uint32_t P = (uint32_t)pop_plane(d.nx, d.ny);
  gcchar *b0 = (gcchar *)(d.src + (size_t)P * (size_t)Z);
  gcchar *b1 = b0 + (size_t)(19 * kBN * 4);
  uint32_t px[3], py[3];
  px[0] = brick_x(X == 0 ? d.nx - 1 : X - 1);
  px[1] = brick_x(X);
  px[2] = brick_x(X == d.nx - 1 ? 0 : X + 1);
  py[0] = brick_y(Y == 0 ? d.ny - 1 : Y - 1, d.nx);
  py[1] = brick_y(Y, d.nx);
  py[2] = brick_y(Y == d.ny - 1 ? 0 : Y + 1, d.nx);
  // The offsets do not depend on Z (the base does), so a z-marching loop
  // would otherwise keep all 38 of them live in registers across planes;
  // these opaque moves make them cheap per-plane arithmetic instead.
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    asm volatile("" : "+v"(px[i]));
    asm volatile("" : "+v"(py[i]));
  }
  const uint32_t own = P + py[1] + px[1];
  pull_rec<0>(b0, b1, m, own, P, py, px, v);
}

// Type of the density sums.  Populations are stored in FP32 (the HBM
// bytes); the 19-term density sums are FP64 (see collide() for the rest).
typedef double acc_t;

__device__ __forceinline__ acc_t sum19(const float (&a)[19]) {
  acc_t s = 0;
#pragma unroll
  for (int k = 0; k < 19; ++k) s += (acc_t)a[k];
  return s;
}

// Density seen by the interaction sums at (X, Y, Z): zero on solid nodes and
// beyond walls, the imposed value on bath nodes, Eq. 2 on fluid nodes.  With
// KEEP, the pulled populations, the mask word and the two FP64 sums of the
// shifted populations (zero unless the node is fluid) are returned for the
// collision of this node.
template <bool KEEP>
__device__ __forceinline__ float2 density_at(const Dom &d, const Phys &P, int X, int Y, int Z,
                                             float (&v)[2][19], uint32_t &mword,
                                             double (&ds)[2]) {
  if (KEEP) ds[0] = ds[1] = 0.0;
  const long long n = node_of(d, X, Y, Z);
  if (n < 0) {
    if (KEEP) mword = kSolid << kTypeShift;
    return make_float2(0.f, 0.f);
  }
  const uint32_t m = d.mask[n];
  if (KEEP) mword = m;
  const uint32_t t = m >> kTypeShift;
  if (t == kSolid) return make_float2(0.f, 0.f);
  if (t == kResIn) return make_float2(P.rres[0][0], P.rres[0][1]);
  if (t == kResOut) return make_float2(P.rres[1][0], P.rres[1][1]);
  int X2 = wrap(X, d.nx), Y2 = wrap(Y, d.ny), Z2 = wrap(Z, d.nz);
  if (KEEP) {
    pull(d, m, X2, Y2, Z2, v);
    ds[0] = sum19(v[0]);
    ds[1] = sum19(v[1]);
    return make_float2((float)((acc_t)P.rho_ref + ds[0]), (float)((acc_t)P.rho_ref + ds[1]));
  } else {
    float t2[2][19];
    pull(d, m, X2, Y2, Z2, t2);
    return make_float2((float)((acc_t)P.rho_ref + sum19(t2[0])), (float)((acc_t)P.rho_ref + sum19(t2[1])));
  }
}

// BGK collision of one fluid node (Eq. 1 right-hand side) with the cohesion
// force of Eq. 4 (S = sum_k w_k rho(x + e_k) e_k of each component, from the
// density stencil) and the adhesion force toward solid neighbours, entering
// through the velocity shift u_eq = u' + tau F / rho.  v: pulled shifted
// populations in, post-collision shifted populations out.
//
// Precision: the densities (sum of the 19 populations) and the post-collision
// rest population are FP64; momenta, forces, velocities and the 18 moving
// equilibria are FP32.  The rest population is set to the FP64 density minus
// the 18 moving post-collision values, so the collision conserves each
// component's mass to FP64 rounding (the BGK update does so exactly), and
// FP32 rounding of the weights (their FP32 sum is not exactly 1) cannot bias
// the mass step after step.  Momenta are summed from opposite-pair
// differences.  drd: the FP64 sums of each component's 19 shifted
// populations, as density_at() took them when the node was pulled.
__device__ __forceinline__ void collide(const Phys &P, uint32_t m, const float (&Sw)[3],
                                        const float (&Sn)[3], const double (&drd)[2],
                                        float (&v)[2][19]) {
  float dr[2], rho[2], j[2][3];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    dr[c] = (float)drd[c];
    rho[c] = (float)((double)P.rho_ref + drd[c]);
    float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      if (k > opp(k)) continue;
      const float dk = v[c][k] - v[c][opp(k)];
      if (ex(k)) jx += ex(k) > 0 ? dk : -dk;
      if (ey(k)) jy += ey(k) > 0 ? dk : -dk;
      if (ez(k)) jz += ez(k) > 0 ? dk : -dk;
    }
    j[c][0] = jx;
    j[c][1] = jy;
    j[c][2] = jz;
  }
  // adhesion direction: zero (the same +0 the sum gives) when no link is cut
  float A[3] = {0.f, 0.f, 0.f};
  if ((m & kLinkBits) != 0u)
#pragma unroll
  for (int k = 1; k < 19; ++k) {
    const float s = (float)((m >> opp(k)) & 1u) * wf(k);
    if (ex(k)) A[0] += ex(k) > 0 ? s : -s;
    if (ey(k)) A[1] += ey(k) > 0 ? s : -s;
    if (ez(k)) A[2] += ez(k) > 0 ? s : -s;
  }
  float F[2][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    F[0][a] = -P.G * rho[0] * Sn[a] - P.Gads[0] * rho[0] * A[a];
    F[1][a] = -P.G * rho[1] * Sw[a] - P.Gads[1] * rho[1] * A[a];
  }
  const float it0 = P.itau[0], it1 = P.itau[1];
  const float den = rho[0] * it0 + rho[1] * it1;
  // quotients as products with three reciprocals (the node-list path below
  // takes the same ones, so both paths stay bit-identical)
  const float iden = 1.0f / den;
  float up[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) up[a] = (j[0][a] * it0 + j[1][a] * it1) * iden;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    float u[3];
    const float tc = P.tau[c], itc = P.itau[c];
    const float irho = 1.0f / rho[c];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = up[a] + tc * F[c][a] * irho;
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double rest = drd[c];
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      float eu = 0.f;
      if (ex(k)) eu += ex(k) > 0 ? u[0] : -u[0];
      if (ey(k)) eu += ey(k) > 0 ? u[1] : -u[1];
      if (ez(k)) eu += ez(k) > 0 ? u[2] : -u[2];
      const float geq = wf(k) * (dr[c] + rho[c] * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
      const float g = v[c][k];
      const float gs = g - (g - geq) * itc;
      v[c][k] = gs;
      rest -= (double)gs;
    }
    v[c][0] = (float)rest;
  }
}

// Store the post-collision populations of the node at (X, Y, Z) (the ghost
// planes of z-periodic subdomains are refreshed by k_ghost after the step).
__device__ __forceinline__ void store_node(const Dom &d, int X, int Y, int Z,
                                           const float (&v)[2][19]) {
  const size_t P = pop_plane(d.nx, d.ny);
  uint32_t own = brick_y(Y, d.nx) + brick_x(X);
  asm volatile("" : "+v"(own));  // per-plane offsets, as in pull()
  gchar *b = (gchar *)(d.dst + P * (size_t)(Z + 1));
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < 19; ++k)
      __builtin_nontemporal_store(
          v[c][k], (__attribute__((address_space(1))) float *)(
                       b + (size_t)((own + (uint32_t)((19 * c + k) * kBN)) * 4u)));
}

// ---- fused step ------------------------------------------------------------
// A workgroup owns a TX x TY column of nodes and marches it through a
// z-segment, software-pipelined over three planes.  Entering iteration Z, the
// thread holds its own node of plane Z in registers, its node of plane Z+1 in
// a private LDS slot, and the LDS density ring holds planes Z-1..Z+1.  It
//   1. issues the pulls of plane Z+2 for its halo node and its own node,
//   2. sums the halo pull into the ring (plane Z+2),
//   3. collides plane Z with the 18-neighbour density stencil while the own
//      pull is still in flight, and stores it,
//   4. sums the own pull into the ring, rotates plane Z+1 from LDS into
//      registers and parks plane Z+2 in LDS,
//   5. synchronises the workgroup.
// Every population is read from memory once per step (halo pulls re-read
// neighbour tiles' lines, which are normally still in L2).
template <int TX, int TY>
__device__ __forceinline__ void halo_slot(int h, int &hx, int &hy) {
  constexpr int HR = 2 * (TX + 2);
  if (h < HR) {
    hx = h % (TX + 2) - 1;
    hy = h < TX + 2 ? -1 : TY;
  } else {
    const int u = h - HR;
    hx = u < TY ? -1 : TX;
    hy = u % TY;
  }
}

// At most 168 VGPRs per lane: three waves per SIMD, which the z-march needs
// to keep enough pulls in flight.
template <int TX, int TY>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(3))) void k_step(
    const Throat *__restrict__ throats,
                                                 const TileRef *__restrict__ tiles, int ntiles,
                                                 int parity) {
  constexpr int NT = TX * TY;
  constexpr int H = 2 * (TX + 2) + 2 * TY;  // halo ring of one plane
  static_assert(NT >= H, "tile too small for its halo");
  __shared__ float2 ring[4][TY + 2][TX + 2];
  __shared__ float stage[38][NT];
  __shared__ uint32_t stage_m[NT];

  // lanes follow the storage bricks: 32 consecutive lanes own one 8 x 4
  // brick, so each population load or store of a wavefront is whole lines
  static_assert(TX % kBX == 0 && TY % kBY == 0, "tiles are whole bricks");
  const int tid = threadIdx.x;
  const int tb = tid / kBN;
  const int tx = (tb % (TX / kBX)) * kBX + tid % kBX;
  const int ty = (tb / (TX / kBX)) * kBY + (tid / kBX) % kBY;
  // list entries are handed out so that each XCD (blocks b = xcd mod 8) gets
  // one contiguous range of the tile list, keeping spatial neighbours in one L2
  const int b = blockIdx.x;
  const int q = ntiles >> 3, r = ntiles & 7, xcd = b & 7, idx = b >> 3;
  const TileRef tr = tiles[xcd * q + min(xcd, r) + idx];
  const Throat &T = throats[tr.throat];
  if (!T.active) return;
  Dom d;
  d.src = T.g[parity];
  d.dst = T.g[parity ^ 1];
  d.mask = T.mask;
  d.N = T.N;
  d.nx = T.nx;
  d.ny = T.ny;
  d.nz = T.nz;
  d.per = T.per;
  const Phys P = T.P;
  const int ntx = T.ntx, nty = T.nty, lz = T.lz;
  const int tix = tr.tile % ntx, tiy = (tr.tile / ntx) % nty, tiz = tr.tile / (ntx * nty);
  const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * lz;
  const int z1 = min(z0 + lz, d.nz);
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < d.nx && y < d.ny;
  // the first H threads also pull one halo node each (the halo instructions
  // are then issued by as few wavefronts as possible)
  const bool halo = tid < H;
  int hx = 0, hy = 0;
  if (halo) halo_slot<TX, TY>(tid, hx, hy);

  float cur[2][19], nxt[2][19], hv[2][19];
  uint32_t mcur = 0, mnxt = 0, mh;
  // FP64 population sums of the own node at planes Z, Z+1, Z+2 (for collide)
  double dcur[2], dmid[2], dnxt[2], dh[2];

  // prologue: densities of planes z0-1 .. z0+1, populations of z0 and z0+1
  ring[(z0 - 1) & 3][ty + 1][tx + 1] = density_at<false>(d, P, x, y, z0 - 1, hv, mh, dh);
  if (halo) ring[(z0 - 1) & 3][hy + 1][hx + 1] = density_at<false>(d, P, x0 + hx, y0 + hy, z0 - 1, hv, mh, dh);
  ring[z0 & 3][ty + 1][tx + 1] = density_at<true>(d, P, x, y, z0, cur, mcur, dcur);
  if (halo) ring[z0 & 3][hy + 1][hx + 1] = density_at<false>(d, P, x0 + hx, y0 + hy, z0, hv, mh, dh);
  ring[(z0 + 1) & 3][ty + 1][tx + 1] = density_at<true>(d, P, x, y, z0 + 1, nxt, mnxt, dmid);
  if (halo) ring[(z0 + 1) & 3][hy + 1][hx + 1] = density_at<false>(d, P, x0 + hx, y0 + hy, z0 + 1, hv, mh, dh);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < 19; ++k) stage[c * 19 + k][tid] = nxt[c][k];
  stage_m[tid] = mnxt;
  __syncthreads();

  for (int Z = z0; Z < z1; ++Z) {
    const bool ahead = Z + 2 <= z1;  // plane Z+2 is needed (density halo or next own)
    // 1-2. halo node of plane Z+2, then own node of plane Z+2 (left in flight)
    if (ahead && halo)
      ring[(Z + 2) & 3][hy + 1][hx + 1] = density_at<false>(d, P, x0 + hx, y0 + hy, Z + 2, hv, mh, dh);
    float2 rho_ahead = make_float2(0.f, 0.f);
    dnxt[0] = dnxt[1] = 0.0;
    if (ahead) rho_ahead = density_at<true>(d, P, x, y, Z + 2, nxt, mnxt, dnxt);
    // 3. collide plane Z
    if (own) {
      const uint32_t t = mcur >> kTypeShift;
      if (t == kFluid) {
        float Sw[3] = {0, 0, 0}, Sn[3] = {0, 0, 0};
#pragma unroll
        for (int k = 1; k < 19; ++k) {
          const float2 rn = ring[(Z + ez(k)) & 3][ty + 1 + ey(k)][tx + 1 + ex(k)];
          const float a = wf(k) * rn.x, bb = wf(k) * rn.y;
          if (ex(k)) { Sw[0] += ex(k) > 0 ? a : -a; Sn[0] += ex(k) > 0 ? bb : -bb; }
          if (ey(k)) { Sw[1] += ey(k) > 0 ? a : -a; Sn[1] += ey(k) > 0 ? bb : -bb; }
          if (ez(k)) { Sw[2] += ez(k) > 0 ? a : -a; Sn[2] += ez(k) > 0 ? bb : -bb; }
        }
        collide(P, mcur, Sw, Sn, dcur, cur);
        store_node(d, x, y, Z, cur);
      } else if (t == kResIn || t == kResOut) {
        const int i = t == kResIn ? 0 : 1;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int k = 0; k < 19; ++k) cur[c][k] = wf(k) * P.gres[i][c];
        store_node(d, x, y, Z, cur);
      }
    }
    // 4. publish plane Z+2, rotate Z+1 -> registers, Z+2 -> LDS
    if (ahead) ring[(Z + 2) & 3][ty + 1][tx + 1] = rho_ahead;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < 19; ++k) {
        cur[c][k] = stage[c * 19 + k][tid];
        stage[c * 19 + k][tid] = nxt[c][k];
      }
    mcur = stage_m[tid];
    stage_m[tid] = mnxt;
    dcur[0] = dmid[0];
    dcur[1] = dmid[1];
    dmid[0] = dnxt[0];
    dmid[1] = dnxt[1];
    // 5.
    __syncthreads();
  }
}

// ---- node-list path ---------------------------------------------------------
// For subdomains where most nodes are solid (thin throat prisms, small
// throats) the tiles above spend their lanes on solid nodes.  Here every
// non-solid node of the list (each entry: node index and mask word) gets a
// pair of adjacent lanes, lane c handling component c: a first pass writes
// each node's densities (the same FP64 sums rounded to FP32 that the tiles
// keep in LDS), the second pulls, takes the 18-neighbour stencil of the
// other component's density from that array (zero where the node's link
// bits mark a solid neighbour or a wall), collides and stores.  The pair
// swaps its density and momentum by lane shuffle, so each lane evaluates the
// collision's shared terms from the same operands in the same order as the
// one-lane collide(): results are bit-identical to the tiled step.  A pair
// per node doubles the wavefronts of a small subdomain (a 96^3 throat has
// about one wavefront of nodes per SIMD) and halves each lane's chain of
// loads and arithmetic.  Per fluid node the second pass moves the same 304
// bytes as the fused step plus the stencil reads, the first pass another
// 152 + 8, and each pass reads the 8-byte list entry.
__device__ __forceinline__ const TileRef &list_ref(const TileRef *__restrict__ tiles, int ntiles) {
  const int b = blockIdx.x;
  const int q = ntiles >> 3, r = ntiles & 7, xcd = b & 7, idx = b >> 3;
  return tiles[xcd * q + min(xcd, r) + idx];
}

__device__ __forceinline__ Dom list_dom(const Throat &T, int parity) {
  Dom d;
  d.src = T.g[parity];
  d.dst = T.g[parity ^ 1];
  d.mask = T.mask;
  d.N = T.N;
  d.nx = T.nx;
  d.ny = T.ny;
  d.nz = T.nz;
  d.per = T.per;
  return d;
}

// one component's half of pull(): the 19 populations of component c
template <int K>
__device__ __forceinline__ void pull1_rec(gcchar *b, uint32_t m, uint32_t own, uint32_t P,
                                          const uint32_t (&py)[3], const uint32_t (&px)[3],
                                          float (&v)[19]) {
  constexpr int o = opp(K);
  const bool cut = (m >> K) & 1u;
  const uint32_t off =
      cut ? own + (uint32_t)(o * kBN) : src_index<K>(P, py, px) + (uint32_t)(K * kBN);
  v[K] = *(const __attribute__((address_space(1))) float *)(b + (size_t)(off * 4u));
  if constexpr (K + 1 < 19) pull1_rec<K + 1>(b, m, own, P, py, px, v);
}

__device__ __forceinline__ void pull1(const Dom &d, uint32_t m, int X, int Y, int Z, int c,
                                      float (&v)[19]) {
  const uint32_t P = (uint32_t)pop_plane(d.nx, d.ny);
  gcchar *b = (gcchar *)(d.src + (size_t)P * (size_t)Z) + (size_t)(c * 19 * kBN * 4);
  uint32_t px[3], py[3];
  px[0] = brick_x(X == 0 ? d.nx - 1 : X - 1);
  px[1] = brick_x(X);
  px[2] = brick_x(X == d.nx - 1 ? 0 : X + 1);
  py[0] = brick_y(Y == 0 ? d.ny - 1 : Y - 1, d.nx);
  py[1] = brick_y(Y, d.nx);
  py[2] = brick_y(Y == d.ny - 1 ? 0 : Y + 1, d.nx);
  const uint32_t own = P + py[1] + px[1];
  pull1_rec<0>(b, m, own, P, py, px, v);
}

__device__ __forceinline__ void store1(const Dom &d, int X, int Y, int Z, int c,
                                       const float (&v)[19]) {
  const size_t P = pop_plane(d.nx, d.ny);
  const uint32_t own = brick_y(Y, d.nx) + brick_x(X) + (uint32_t)(19 * c * kBN);
  gchar *b = (gchar *)(d.dst + P * (size_t)(Z + 1));
#pragma unroll
  for (int k = 0; k < 19; ++k)
    __builtin_nontemporal_store(
        v[k], (__attribute__((address_space(1))) float *)(
                  b + (size_t)((own + (uint32_t)(k * kBN)) * 4u)));
}

__device__ __forceinline__ void list_coords(const Dom &d, uint32_t n, int &X, int &Y, int &Z) {
  const uint32_t nx = (uint32_t)d.nx, nxy = nx * (uint32_t)d.ny;
  Z = (int)(n / nxy);
  Y = (int)((n - (uint32_t)Z * nxy) / nx);
  X = (int)(n - (uint32_t)Z * nxy - (uint32_t)Y * nx);
}

__global__ void k_list_entries(const uint32_t *ids, const uint32_t *mask, uint32_t n, uint2 *out) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = make_uint2(ids[i], mask[ids[i]]);
}

hipError_t launch_list_entries(const uint32_t *ids, const uint32_t *mask, uint32_t n, uint2 *out,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<uint32_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_list_entries, dim3(blocks), dim3(256), 0, st, ids, mask, n, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kListBlock) void k_dens_list(const Throat *__restrict__ throats,
                                                          const TileRef *__restrict__ tiles,
                                                          int ntiles, int parity) {
  const TileRef tr = list_ref(tiles, ntiles);
  const Throat &T = throats[tr.throat];
  if (!T.active) return;
  const uint32_t i = (uint32_t)tr.tile * kListNodes + threadIdx.x / 2;
  const int c = threadIdx.x & 1;
  if (i >= T.nlist) return;
  const Dom d = list_dom(T, parity);
  const Phys &P = T.P;
  const uint2 e = T.list[i];
  const uint32_t n = e.x, m = e.y;
  const uint32_t t = m >> kTypeShift;
  float r;
  if (t == kFluid) {
    int X, Y, Z;
    list_coords(d, n, X, Y, Z);
    float v[19];
    pull1(d, m, X, Y, Z, c, v);
    r = (float)((acc_t)P.rho_ref + sum19(v));
  } else {
    r = P.rres[t == kResIn ? 0 : 1][c];
  }
  reinterpret_cast<float *>(T.rho)[2 * (size_t)n + c] = r;
}

__global__ __launch_bounds__(kListBlock) void k_step_list(const Throat *__restrict__ throats,
                                                          const TileRef *__restrict__ tiles,
                                                          int ntiles, int parity) {
  const TileRef tr = list_ref(tiles, ntiles);
  const Throat &T = throats[tr.throat];
  if (!T.active) return;
  const uint32_t i = (uint32_t)tr.tile * kListNodes + threadIdx.x / 2;
  const int c = threadIdx.x & 1;
  if (i >= T.nlist) return;  // both lanes of a pair leave together
  const Dom d = list_dom(T, parity);
  const Phys &P = T.P;
  const uint2 e = T.list[i];
  const uint32_t n = e.x, m = e.y;
  const uint32_t t = m >> kTypeShift;
  int X, Y, Z;
  list_coords(d, n, X, Y, Z);
  float v[19];
  if (t == kFluid) {
    pull1(d, m, X, Y, Z, c, v);
    // stencil of the other component's density (the cohesion of Eq. 4)
    // Neighbour x + e_k is the pull source of direction opp(k): its link bit
    // says whether it is solid or beyond a wall (density zero); otherwise it
    // is in the box or across a periodic face.
    const float *rho_o = reinterpret_cast<const float *>(T.rho) + (1 - c);
    const int xm = X == 0 ? d.nx - 1 : X - 1, xp = X == d.nx - 1 ? 0 : X + 1;
    const int ym = Y == 0 ? d.ny - 1 : Y - 1, yp = Y == d.ny - 1 ? 0 : Y + 1;
    const int zm = Z == 0 ? d.nz - 1 : Z - 1, zp = Z == d.nz - 1 ? 0 : Z + 1;
    float So[3] = {0, 0, 0};
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      const int xn = ex(k) > 0 ? xp : (ex(k) < 0 ? xm : X);
      const int yn = ey(k) > 0 ? yp : (ey(k) < 0 ? ym : Y);
      const int zn = ez(k) > 0 ? zp : (ez(k) < 0 ? zm : Z);
      const uint32_t nb = ((uint32_t)zn * (uint32_t)d.ny + (uint32_t)yn) * (uint32_t)d.nx +
                          (uint32_t)xn;
      const float a = wf(k) * (((m >> opp(k)) & 1u) ? 0.f : rho_o[2 * (size_t)nb]);
      if (ex(k)) So[0] += ex(k) > 0 ? a : -a;
      if (ey(k)) So[1] += ey(k) > 0 ? a : -a;
      if (ez(k)) So[2] += ez(k) > 0 ? a : -a;
    }
    // collide(), one component per lane
    const double drd = sum19(v);
    const float dr = (float)drd;
    const float rho = (float)((double)P.rho_ref + drd);
    float j[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      if (k > opp(k)) continue;
      const float dk = v[k] - v[opp(k)];
      if (ex(k)) j[0] += ex(k) > 0 ? dk : -dk;
      if (ey(k)) j[1] += ey(k) > 0 ? dk : -dk;
      if (ez(k)) j[2] += ez(k) > 0 ? dk : -dk;
    }
    const float rho_p = __shfl_xor(rho, 1);
    float jp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) jp[a] = __shfl_xor(j[a], 1);
    const float rho0 = c == 0 ? rho : rho_p, rho1 = c == 0 ? rho_p : rho;
    float A[3] = {0.f, 0.f, 0.f};
    if ((m & kLinkBits) != 0u)
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      const float s = (float)((m >> opp(k)) & 1u) * wf(k);
      if (ex(k)) A[0] += ex(k) > 0 ? s : -s;
      if (ey(k)) A[1] += ey(k) > 0 ? s : -s;
      if (ez(k)) A[2] += ez(k) > 0 ? s : -s;
    }
    const float gads = P.Gads[c];
    float F[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = -P.G * rho * So[a] - gads * rho * A[a];
    const float it0 = P.itau[0], it1 = P.itau[1];
    const float den = rho0 * it0 + rho1 * it1;
    const float iden = 1.0f / den;
    float up[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float j0 = c == 0 ? j[a] : jp[a], j1 = c == 0 ? jp[a] : j[a];
      up[a] = (j0 * it0 + j1 * it1) * iden;
    }
    const float tc = P.tau[c], itc = P.itau[c];
    const float irho = 1.0f / rho;
    float u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = up[a] + tc * F[a] * irho;
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double rest = drd;
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      float eu = 0.f;
      if (ex(k)) eu += ex(k) > 0 ? u[0] : -u[0];
      if (ey(k)) eu += ey(k) > 0 ? u[1] : -u[1];
      if (ez(k)) eu += ez(k) > 0 ? u[2] : -u[2];
      const float geq = wf(k) * (dr + rho * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
      const float g = v[k];
      const float gs = g - (g - geq) * itc;
      v[k] = gs;
      rest -= (double)gs;
    }
    v[0] = (float)rest;
  } else {
    const int b = t == kResIn ? 0 : 1;
#pragma unroll
    for (int k = 0; k < 19; ++k) v[k] = wf(k) * P.gres[b][c];
  }
  store1(d, X, Y, Z, c, v);
}

bool schedule_valid(const Sched &s) {
  if (s.tx == kListTx) return true;  // node-list path
  // (64, 8) and (32, 16) would need 2 x 78 KB of LDS staging: not offered
  if (s.lz < 1) return false;
  for (int i = 0; i < kNumShapes; ++i)
    if (s.tx == kShapes[i][0] && s.ty == kShapes[i][1]) return true;
  return false;
}

template <int TX, int TY>
static hipError_t step_as(const Throat *th, const TileRef *tiles, int ntiles, int parity,
                          hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_step<TX, TY>), dim3((unsigned)ntiles), dim3(TX * TY), 0, st, th, tiles,
                     ntiles, parity);
  return hipGetLastError();
}

// Ghost planes of z-periodic subdomains after a step: plane 0 of the new
// state is copied to plane nz, plane nz - 1 to plane -1 (two contiguous runs
// of one padded plane each).  Grid: x over the run, y over the listed subdomains.
__global__ __launch_bounds__(256) void k_ghost(const Throat *__restrict__ throats,
                                               const int *__restrict__ ids, int parity) {
  const Throat &T = throats[ids[blockIdx.y]];
  if (!T.active) return;
  float *g = T.g[parity ^ 1];
  const size_t P = pop_plane(T.nx, T.ny);
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < P; i += (size_t)gridDim.x * 256) {
    g[P * (size_t)(T.nz + 1) + i] = g[P + i];
    g[i] = g[P * (size_t)T.nz + i];
  }
}

static hipError_t step_body(const Throat *th, const TileRef *tiles, int ntiles, int tx, int ty,
                            int parity, hipStream_t st) {
  if (tx == kListTx) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dens_list, dim3((unsigned)ntiles), dim3(kListBlock), 0, st, th, tiles,
                       ntiles, parity);
    hipLaunchKernelGGL(k_step_list, dim3((unsigned)ntiles), dim3(kListBlock), 0, st, th, tiles,
                       ntiles, parity);
    return hipGetLastError();
  }
  if (tx == 32) {
    if (ty == 4) return step_as<32, 4>(th, tiles, ntiles, parity, st);
    return step_as<32, 8>(th, tiles, ntiles, parity, st);
  }
  if (tx == 16) {
    if (ty == 4) return step_as<16, 4>(th, tiles, ntiles, parity, st);
    return step_as<16, 8>(th, tiles, ntiles, parity, st);
  }
  if (tx == 8) return step_as<8, 8>(th, tiles, ntiles, parity, st);
  return step_as<64, 4>(th, tiles, ntiles, parity, st);
}

hipError_t launch_step(const Throat *th, const TileRef *tiles, int ntiles, int tx, int ty,
                       int parity, hipStream_t st, const int *zper_ids, int n_zper) {
  if (!schedule_valid(Sched{tx, ty, 1})) return hipErrorInvalidValue;
  const hipError_t e = step_body(th, tiles, ntiles, tx, ty, parity, st);
  if (e != hipSuccess || n_zper <= 0 || ntiles <= 0) return e;
  hipLaunchKernelGGL(k_ghost, dim3(1024, (unsigned)n_zper), dim3(256), 0, st, th, zper_ids, parity);
  return hipGetLastError();
}

void brick_map(const uint8_t *types, int nx, int ny, int nz, std::vector<uint8_t> &live,
               size_t &nonsolid) {
  // 8 x 4 patches of the tile grid (tiles start at multiples of their
  // sides, which are multiples of 8 and 4), whatever the storage bricks' offset
  const int nbx = (nx + kBX - 1) / kBX, nby = (ny + kBY - 1) / kBY;
  live.assign((size_t)nbx * nby * nz, 0);
  nonsolid = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      const uint8_t *row = types + (size_t)nx * ((size_t)y + (size_t)ny * z);
      uint8_t *b = live.data() + (size_t)nbx * ((size_t)(y / kBY) + (size_t)nby * z);
      for (int x = 0; x < nx; ++x)
        if (row[x] != kSolid) {
          b[x / kBX] = 1;
          ++nonsolid;
        }
    }
}

void list_tiles(const uint8_t *live, size_t nonsolid, int nx, int ny, int nz, int tx, int ty,
                int lz, int throat, std::vector<TileRef> &out) {
  if (tx == kListTx) {  // node-list path: chunks of kListNodes non-solid nodes
    for (size_t c = 0; c * kListNodes < nonsolid; ++c) out.push_back(TileRef{throat, (int)c});
    return;
  }
  const int nbx = (nx + kBX - 1) / kBX, nby = (ny + kBY - 1) / kBY;
  const int bpx = tx / kBX, bpy = ty / kBY;  // patches per tile side
  const int ntx = (nx + tx - 1) / tx, nty = (ny + ty - 1) / ty, ntz = (nz + lz - 1) / lz;
  // liveness of each (x-tile, y-tile) cell of every plane, then of every z-segment
  std::vector<uint8_t> cell((size_t)ntx * nty * nz, 0);
  for (int z = 0; z < nz; ++z)
    for (int by = 0; by < nby; ++by) {
      const uint8_t *b = live + (size_t)nbx * ((size_t)by + (size_t)nby * z);
      uint8_t *c = cell.data() + (size_t)ntx * ((size_t)(by / bpy) + (size_t)nty * z);
      for (int bx = 0; bx < nbx; ++bx)
        if (b[bx]) c[bx / bpx] = 1;
    }
  for (int tz = 0; tz < ntz; ++tz)
    for (int tyi = 0; tyi < nty; ++tyi)
      for (int txi = 0; txi < ntx; ++txi) {
        bool any = false;
        for (int z = tz * lz; z < std::min(nz, (tz + 1) * lz) && !any; ++z)
          any = cell[(size_t)txi + (size_t)ntx * ((size_t)tyi + (size_t)nty * z)] != 0;
        if (any) out.push_back(TileRef{throat, txi + ntx * (tyi + nty * tz)});
      }
}

// ---- geometry ----------------------------------------------------------------
// Node classes from spheres and the prism closure (predicates in geom.h).
// Spheres are binned on the host into cubic cells of kVoxCell nodes: a node
// tests only the spheres whose bounding box (widened by one node) meets its
// cell, in increasing sphere order, which classifies every node exactly as
// testing all spheres would.
__global__ void k_voxelize(const double *sph, const VoxBins bins, int prism, int i0, int i1,
                           int i2, int nx, int ny, int nz, int res_z, uint8_t *types) {
  const size_t N = (size_t)nx * ny * nz;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((size_t)nx * ny));
    const int c = x / kVoxCell + bins.ncx * (y / kVoxCell + bins.ncy * (z / kVoxCell));
    bool solid = false;
    for (int j = bins.start[c]; j < bins.start[c + 1] && !solid; ++j)
      solid = geom::in_sphere(x, y, z, sph + 4 * bins.ids[j]);
    if (!solid && prism) solid = !geom::in_prism(sph + 4 * i0, sph + 4 * i1, sph + 4 * i2, x, y);
    uint8_t t = kFluid;
    if (solid) t = kSolid;
    else if (res_z && z == 0) t = kResIn;
    else if (res_z && z == nz - 1) t = kResOut;
    types[n] = t;
  }
}

void bin_spheres(const double *sph, int ns, int nx, int ny, int nz, std::vector<int> &start,
                 std::vector<int> &ids, int &ncx, int &ncy, int &ncz) {
  ncx = (nx + kVoxCell - 1) / kVoxCell;
  ncy = (ny + kVoxCell - 1) / kVoxCell;
  ncz = (nz + kVoxCell - 1) / kVoxCell;
  const int nn[3] = {nx, ny, nz};
  std::vector<std::vector<int>> cell((size_t)ncx * ncy * ncz);
  for (int i = 0; i < ns; ++i) {
    int lo[3], hi[3];
    bool empty = false;
    for (int a = 0; a < 3; ++a) {
      const double l = std::floor(sph[4 * i + a] - sph[4 * i + 3]) - 1.0;
      const double h = std::ceil(sph[4 * i + a] + sph[4 * i + 3]) + 1.0;
      if (h < 0.0 || l > nn[a] - 1.0) empty = true;
      lo[a] = (int)std::max(0.0, l) / kVoxCell;
      hi[a] = (int)std::min((double)(nn[a] - 1), h) / kVoxCell;
    }
    if (empty) continue;
    for (int cz = lo[2]; cz <= hi[2]; ++cz)
      for (int cy = lo[1]; cy <= hi[1]; ++cy)
        for (int cx = lo[0]; cx <= hi[0]; ++cx)
          cell[(size_t)cx + (size_t)ncx * ((size_t)cy + (size_t)ncy * cz)].push_back(i);
  }
  start.assign(cell.size() + 1, 0);
  ids.clear();
  for (size_t c = 0; c < cell.size(); ++c) {
    start[c] = (int)ids.size();
    ids.insert(ids.end(), cell[c].begin(), cell[c].end());
  }
  start[cell.size()] = (int)ids.size();
}

hipError_t launch_voxelize(const double *spheres, const VoxBins &bins, int prism, const int *ids,
                           int nx, int ny, int nz, int res_z, uint8_t *types, hipStream_t st) {
  const size_t N = (size_t)nx * ny * nz;
  const unsigned blocks = (unsigned)std::min<size_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_voxelize, dim3(blocks), dim3(256), 0, st, spheres, bins, prism, ids[0],
                     ids[1], ids[2], nx, ny, nz, res_z, types);
  return hipGetLastError();
}

__global__ void k_links(const uint8_t *types, int nx, int ny, int nz, int per, uint32_t *mask) {
  const size_t N = (size_t)nx * ny * nz;
  Dom d{};
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.per = per;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((size_t)nx * ny));
    uint32_t m = 0;
#pragma unroll
    for (int k = 1; k < 19; ++k) {
      const long long s = node_of(d, x - ex(k), y - ey(k), z - ez(k));
      if (s < 0 || types[s] == kSolid) m |= 1u << k;
    }
    mask[n] = m | ((uint32_t)types[n] << kTypeShift);
  }
}

hipError_t launch_links(const uint8_t *types, int nx, int ny, int nz, int per, uint32_t *mask,
                        hipStream_t st) {
  const size_t N = (size_t)nx * ny * nz;
  const unsigned blocks = (unsigned)std::min<size_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_links, dim3(blocks), dim3(256), 0, st, types, nx, ny, nz, per, mask);
  return hipGetLastError();
}

// ---- initial state ------------------------------------------------------------
// Post-collision values of a virtual step -1 chosen so that the first pull
// yields f(x,0) = f_eq(rho(x,0), u = 0) = w_k rho(x,0) on every fluid node:
// slot k of node y holds w_k rho(y + e_k), or w_k rho(y) when y + e_k is
// solid or beyond a wall (that slot is then only read back by y's own
// bounce-back).
__device__ __forceinline__ double rho0_of(const uint32_t *mask, const double *rho_init,
                                          double maj, double mnr, int z_front, const double *rres,
                                          size_t N, size_t n, int z, int c) {
  const uint32_t t = mask[n] >> kTypeShift;
  if (t == kResIn) return rres[0 * 2 + c];
  if (t == kResOut) return rres[1 * 2 + c];
  if (rho_init) return rho_init[(size_t)c * N + n];
  const bool nw = z <= z_front;
  return (c == 1) == nw ? maj : mnr;
}

__global__ void k_init(Dom d, double rho_ref, const double *rho_init, double maj, double mnr,
                       int z_front, const double *rres, float *g) {
  const size_t P = pop_plane(d.nx, d.ny);
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < d.N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(n % d.nx), y = (int)((n / d.nx) % d.ny), z = (int)(n / ((size_t)d.nx * d.ny));
    // this node's population 0 in its plane and, on a z-periodic subdomain,
    // in the ghost plane that mirrors it
    float *slot = g + P * (size_t)(z + 1) + brick_y(y, d.nx) + brick_x(x);
    float *ghost = nullptr;
    if ((d.per & 4) && z == 0) ghost = slot + P * (size_t)d.nz;
    if ((d.per & 4) && z == d.nz - 1) ghost = slot - P * (size_t)d.nz;
    const uint32_t t = d.mask[n] >> kTypeShift;
    if (t == kSolid) {
      for (int q = 0; q < 38; ++q) {
        slot[(size_t)q * kBN] = 0.f;
        if (ghost) ghost[(size_t)q * kBN] = 0.f;
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      long long tgt = node_of(d, x + ex(k), y + ey(k), z + ez(k));
      if (tgt >= 0 && (d.mask[tgt] >> kTypeShift) == kSolid) tgt = -1;
      const size_t src = tgt < 0 ? n : (size_t)tgt;
      const int zs = (int)(src / ((size_t)d.nx * d.ny));
      for (int c = 0; c < 2; ++c) {
        const double r = rho0_of(d.mask, rho_init, maj, mnr, z_front, rres, d.N, src, zs, c);
        const float gv = (float)(wd(k) * (r - rho_ref));
        slot[(size_t)(c * 19 + k) * kBN] = gv;
        if (ghost) ghost[(size_t)(c * 19 + k) * kBN] = gv;
      }
    }
  }
}

hipError_t launch_init(const Dom &d, const Phys &P, const double *rho_init, double maj, double mnr,
                       int z_front, const double *rres_d, float *g, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<size_t>((d.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, st, d, (double)P.rho_ref, rho_init, maj,
                     mnr, z_front, rres_d, g);
  return hipGetLastError();
}

// ---- read-back: pre-collision populations and densities in FP64 ------------
__global__ void k_export(Dom d, Phys P, const double *rres, double *f) {
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < d.N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(n % d.nx), y = (int)((n / d.nx) % d.ny), z = (int)(n / ((size_t)d.nx * d.ny));
    const uint32_t m = d.mask[n];
    const uint32_t t = m >> kTypeShift;
    float v[2][19];
    if (t == kFluid) pull(d, m, x, y, z, v);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < 19; ++k) {
        double o = 0.0;
        if (t == kFluid) o = wd(k) * (double)P.rho_ref + (double)v[c][k];
        else if (t == kResIn) o = wd(k) * rres[0 * 2 + c];
        else if (t == kResOut) o = wd(k) * rres[1 * 2 + c];
        f[(size_t)(c * 19 + k) * d.N + n] = o;
      }
  }
}

hipError_t launch_export(const Dom &d, const Phys &P, const double *rres_d, double *f,
                         hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<size_t>((d.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_export, dim3(blocks), dim3(256), 0, st, d, P, rres_d, f);
  return hipGetLastError();
}

__global__ void k_density(Dom d, Phys P, const double *rres, double *rho) {
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < d.N;
       n += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(n % d.nx), y = (int)((n / d.nx) % d.ny), z = (int)(n / ((size_t)d.nx * d.ny));
    const uint32_t m = d.mask[n];
    const uint32_t t = m >> kTypeShift;
    double r0 = 0.0, r1 = 0.0;
    if (t == kFluid) {
      float v[2][19];
      pull(d, m, x, y, z, v);
      r0 = (double)(float)((acc_t)P.rho_ref + sum19(v[0]));
      r1 = (double)(float)((acc_t)P.rho_ref + sum19(v[1]));
    } else if (t == kResIn) {
      r0 = rres[0];
      r1 = rres[1];
    } else if (t == kResOut) {
      r0 = rres[2];
      r1 = rres[3];
    }
    rho[n] = r0;
    rho[d.N + n] = r1;
  }
}

hipError_t launch_density(const Dom &d, const Phys &P, const double *rres_d, double *rho,
                          hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<size_t>((d.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_density, dim3(blocks), dim3(256), 0, st, d, P, rres_d, rho);
  return hipGetLastError();
}

// ---- fixed staging array of the allocation-free density read-back ---------
// A file-scope device array, one copy per device for the life of the process.
// Host code never uses its name as an address (on the host the name is only a
// stand-in for the symbol): the device address of the current device's copy
// comes from hipGetSymbolAddress, taken once per device and kept.
static __device__ __align__(256) __attribute__((used)) double scratch[kScratchDoubles];

hipError_t scratch_address(double **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = (double *)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

// ---- FP64 reductions ------------------------------------------------------
// Two passes with a fixed summation order (strided per thread inside a node
// chunk, LDS tree per chunk, then the chunks of a subdomain summed in order
// by one thread), so results are bitwise reproducible and identical whether
// a subdomain is reduced alone or inside a batch.
constexpr int kRedThreads = 256;
constexpr int kRedVals = 3;

void list_chunks(int throat, uint32_t N, std::vector<Chunk> &out) {
  for (uint32_t s = 0; s < N; s += kChunkNodes)
    out.push_back(Chunk{throat, s, std::min(kChunkNodes, N - s)});
}

void list_red_chunks(int throat, uint32_t nlist, std::vector<Chunk> &out) {
  for (uint32_t s = 0; s < nlist; s += kRedEntries)
    out.push_back(Chunk{throat, s, std::min(kRedEntries, nlist - s)});
}

__device__ __forceinline__ void block_sum(double (&v)[kRedVals], double (*sh)[kRedThreads]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kRedVals; ++i) sh[i][t] = v[i];
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int i = 0; i < kRedVals; ++i) sh[i][t] += sh[i][t + s];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kRedVals; ++i) v[i] = sh[i][0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_chunks(const Throat *__restrict__ th,
                                                               const Chunk *__restrict__ chunks,
                                                               const RedInfo *__restrict__ info,
                                                               int parity, double *partials,
                                                               double *probe_out) {
  __shared__ double sh[kRedVals][kRedThreads];
  const Chunk ch = chunks[blockIdx.x];
  const Throat &T = th[ch.throat];
  Dom d;
  d.src = T.g[parity];
  d.dst = nullptr;
  d.mask = T.mask;
  d.N = T.N;
  d.nx = T.nx;
  d.ny = T.ny;
  d.nz = T.nz;
  d.per = T.per;
  const float rho_ref = T.P.rho_ref;
  const RedInfo ri = info[ch.throat];
  double acc[kRedVals] = {0.0, 0.0, 0.0};
  for (uint32_t i = threadIdx.x; i < ch.count; i += kRedThreads) {
    const uint2 e = T.list[ch.start + i];
    const uint32_t n = e.x, m = e.y;
    if ((m >> kTypeShift) != kFluid) continue;
    const int x = (int)(n % (uint32_t)d.nx), y = (int)((n / (uint32_t)d.nx) % (uint32_t)d.ny);
    const int z = (int)(n / ((uint32_t)d.nx * (uint32_t)d.ny));
    float v[2][19];
    pull(d, m, x, y, z, v);
    const double a = (double)(float)((acc_t)rho_ref + sum19(v[0]));
    const double b = (double)(float)((acc_t)rho_ref + sum19(v[1]));
    acc[0] += a;
    acc[1] += b;
    acc[2] += ((a - b) / (a + b) + ri.phib) / (2.0 * ri.phib);
    if ((long long)n == ri.probe) {
      probe_out[2 * ch.throat] = a;
      probe_out[2 * ch.throat + 1] = b;
    }
  }
  block_sum(acc, sh);
  if (threadIdx.x == 0)
    for (int i = 0; i < kRedVals; ++i) partials[(size_t)blockIdx.x * kRedVals + i] = acc[i];
}

__global__ void k_reduce_throats(const int *first, const int *count, int n,
                                 const double *partials, double *sums) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double acc[kRedVals] = {0.0, 0.0, 0.0};
  for (int c = first[t]; c < first[t] + count[t]; ++c)
    for (int i = 0; i < kRedVals; ++i) acc[i] += partials[(size_t)c * kRedVals + i];
  for (int i = 0; i < kRedVals; ++i) sums[(size_t)t * kRedVals + i] = acc[i];
}

hipError_t launch_reduce_chunks(const Throat *th, const Chunk *chunks, int nchunks,
                                const RedInfo *info, int parity, double *partials,
                                double *probe_out, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(nchunks), dim3(kRedThreads), 0, st, th, chunks, info,
                     parity, partials, probe_out);
  return hipGetLastError();
}

hipError_t launch_reduce_throats(const int *first, const int *count, int n, const double *partials,
                                 double *sums, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_throats, dim3((n + 255) / 256), dim3(256), 0, st, first, count, n,
                     partials, sums);
  return hipGetLastError();
}

// ---- device-side drainage ramp (Sec. 2.2.2) ---------------------------------
// The same decisions as the host ramp of a single subdomain, taken for every
// subdomain of a batch between chunks of steps, so that the whole ramp runs
// as graph replays without host decisions per subdomain or per step.
__device__ __forceinline__ void set_inlet(Throat &T, const RampDev &R, double pc) {
  const double rin = R.rho_out + pc / R.dpc_drho;
  T.P.rres[0][1] = (float)rin;
  T.P.gres[0][1] = (float)(rin - R.rho_ref);
}

__global__ void k_ramp_begin(Throat *th, RampDev *rd, const double *pc, RampCfg cfg,
                             const double *sums, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  RampDev R = rd[t];
  const double S = R.n_fluid ? sums[3 * t + 2] / (double)R.n_fluid : 0.0;
  R.phase = kPhaseRamp;
  R.point = 0;
  R.invaded_at = -1;
  R.n_bisect = 0;
  R.warn = 0;
  R.failed = 0;
  R.steps_pt = 0;
  R.total_steps = 0;
  R.S_old = S;
  R.S_stable = S;
  R.stable_pc = 0.0;
  R.req = kSaveStable;
  set_inlet(th[t], R, pc[(size_t)t * cfg.n_pc]);
  th[t].active = 1;
  rd[t] = R;
}

__device__ __forceinline__ void ramp_next_point(Throat &T, RampDev &R, const double *pcs,
                                                const RampCfg &cfg, double S_now) {
  R.point += 1;
  if (R.point >= cfg.n_pc) {
    R.phase = kPhaseDone;
    T.active = 0;
    return;
  }
  set_inlet(T, R, pcs[R.point]);
  R.S_old = S_now;
  R.steps_pt = 0;
}

__device__ __forceinline__ void ramp_trial(Throat &T, RampDev &R) {
  R.mid = 0.5 * (R.lo + R.hi);
  R.req |= kRestoreStable;
  set_inlet(T, R, R.mid);
  R.S_old = R.S_stable;
  R.steps_pt = 0;
}

// a subdomain whose state became non-finite: it stops, and the ramp points
// from `from` on are marked non-finite (none of them gets a result)
__device__ __forceinline__ void ramp_fail(Throat &T, RampDev &R, int *status, int from,
                                          int n_pc) {
  R.failed = 1;
  R.phase = kPhaseDone;
  T.active = 0;
  for (int j = from; j < n_pc; ++j) status[j] = 2;  // LBM_PT_NONFINITE
}

__global__ __launch_bounds__(256) void k_ramp_advance(Throat *th, RampDev *rd, const double *pc,
                                                      RampCfg cfg, const double *sums,
                                                      const double *probe, double *S_out,
                                                      long long *steps_out, int *status_out,
                                                      int n, int *n_active_out) {
  __shared__ int cnt[256];
  int active = 0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    RampDev R = rd[t];
    if (R.phase == kPhaseDone) continue;
    Throat &T = th[t];
    const double *pcs = pc + (size_t)t * cfg.n_pc;
    R.req = 0;  // the previous requests have been carried out
    const double S = R.n_fluid ? sums[3 * t + 2] / (double)R.n_fluid : 0.0;
    const bool inv = probe[2 * t + 1] > probe[2 * t];
    R.steps_pt += cfg.every;
    R.total_steps += cfg.every;
    const bool nonfin = !isfinite(S);
    const bool conv = fabs(S - R.S_old) < cfg.tol;
    if (!nonfin && !conv && R.steps_pt < cfg.cap) {
      R.S_old = S;
      rd[t] = R;
      ++active;
      continue;
    }
    const int st = nonfin ? 2 : (conv ? 0 : 1);
    if (R.phase == kPhaseRamp) {
      const int i = R.point;
      S_out[(size_t)t * cfg.n_pc + i] = S;
      steps_out[(size_t)t * cfg.n_pc + i] = R.steps_pt;
      status_out[(size_t)t * cfg.n_pc + i] = st;
      R.warn |= st == 1;
      if (nonfin) {
        ramp_fail(T, R, status_out + (size_t)t * cfg.n_pc, i + 1, cfg.n_pc);
      } else if (!inv) {
        R.req |= kSaveStable;
        R.S_stable = S;
        R.stable_pc = pcs[i];
        ramp_next_point(T, R, pcs, cfg, S);
      } else if (R.invaded_at >= 0) {
        ramp_next_point(T, R, pcs, cfg, S);
      } else {
        R.invaded_at = i;
        R.lo = i == 0 ? 0.0 : R.stable_pc;
        R.hi = pcs[i];
        if ((R.hi - R.lo) / R.hi > cfg.rel) {
          R.req |= kSaveMain;
          R.S_main = S;
          R.rho_in_main = pcs[i];
          R.phase = kPhaseBisect;
          ramp_trial(T, R);
        } else {
          ramp_next_point(T, R, pcs, cfg, S);
        }
      }
    } else {  // bisection run finished
      R.n_bisect += 1;
      if (nonfin) {
        // the ramp point being bisected keeps its status; the points after
        // it are never reached
        ramp_fail(T, R, status_out + (size_t)t * cfg.n_pc, R.point + 1, cfg.n_pc);
      } else {
        if (inv) {
          R.hi = R.mid;
        } else {
          R.lo = R.mid;
          R.req |= kSaveStable;
          R.S_stable = S;
        }
        const bool wide = (R.hi - R.lo) / R.hi > cfg.rel;
        if (wide && R.n_bisect < kMaxBisect) {
          ramp_trial(T, R);
        } else {
          R.warn |= wide;
          R.req |= kRestoreMain;
          R.phase = kPhaseRamp;
          ramp_next_point(T, R, pcs, cfg, R.S_main);
        }
      }
    }
    if (R.phase != kPhaseDone) ++active;
    rd[t] = R;
  }
  cnt[threadIdx.x] = active;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) n_active_out[0] = cnt[0];
}

__global__ __launch_bounds__(256) void k_copy_requests(const Throat *__restrict__ th,
                                                       const RampDev *__restrict__ rd,
                                                       const Ckpt *__restrict__ ck,
                                                       const Chunk *__restrict__ chunks,
                                                       int parity) {
  const Chunk c = chunks[blockIdx.x];
  const int req = rd[c.throat].req;
  if (!req) return;
  const Throat &T = th[c.throat];
  float *g = T.g[parity];
  float *sa = ck[c.throat].stable, *ma = ck[c.throat].main;
  // the subdomain's chunks split its whole buffer (ghost planes included)
  // into equal flat ranges, chunk i taking the i-th
  const size_t E = pop_elems(T.nx, T.ny, T.nz);
  const size_t nch = (T.N + kChunkNodes - 1) / kChunkNodes;
  const size_t len = (E + nch - 1) / nch;
  const size_t lo = (size_t)(c.start / kChunkNodes) * len;
  const size_t hi = lo + len < E ? lo + len : E;
  for (size_t o = lo + threadIdx.x; o < hi; o += blockDim.x) {
    const float v = g[o];
    if (req & kSaveStable) sa[o] = v;
    if (req & kSaveMain) ma[o] = v;
    if (req & kRestoreStable) g[o] = sa[o];
    if (req & kRestoreMain) g[o] = ma[o];
  }
}

hipError_t launch_ramp_begin(Throat *th, RampDev *rd, const double *pc, const RampCfg &cfg,
                             const double *sums, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_ramp_begin, dim3((n + 255) / 256), dim3(256), 0, st, th, rd, pc, cfg, sums,
                     n);
  return hipGetLastError();
}

hipError_t launch_ramp_advance(Throat *th, RampDev *rd, const double *pc, const RampCfg &cfg,
                               const double *sums, const double *probe, double *S_out,
                               long long *steps_out, int *status_out, int n, int *n_active_out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_ramp_advance, dim3(1), dim3(256), 0, st, th, rd, pc, cfg, sums, probe,
                     S_out, steps_out, status_out, n, n_active_out);
  return hipGetLastError();
}

hipError_t launch_copy_requests(const Throat *th, const RampDev *rd, const Ckpt *ck,
                                const Chunk *chunks, int nchunks, int parity, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_requests, dim3(nchunks), dim3(256), 0, st, th, rd, ck, chunks, parity);
  return hipGetLastError();
}

// ---- stream-copy probe: achievable HBM bandwidth on this device ----------
typedef float v4f __attribute__((ext_vector_type(4)));

// one 16-byte element per thread, plain loads and stores (the fastest copy
// form measured on this device)
__global__ __launch_bounds__(256) void k_copy(const v4f *__restrict__ a, v4f *__restrict__ b,
                                              size_t n4) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n4) b[i] = a[i];
}

hipError_t launch_copy(const float *a, float *b, size_t n_floats, hipStream_t st) {
  const size_t n4 = n_floats / 4;
  const size_t blocks = (n4 + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const v4f *)a, (v4f *)b, n4);
  return hipGetLastError();
}

}  // namespace sc
