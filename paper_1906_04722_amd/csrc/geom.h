// geom.h -- geometric predicates shared by the voxelizer and the surrogate's
// occupancy descriptor.  FP64 with every product and sum rounded separately
// (no fused multiply-add), so a point's class does not depend on the
// compiler's contraction choices and matches a plain FP64 evaluation in the
// same order.
#pragma once

#include <hip/hip_runtime.h>

namespace geom {

// |p - c|^2 <= r^2 for a sphere s = (cx, cy, cz, r), summed x, y, z in order
__device__ __forceinline__ bool in_sphere(double x, double y, double z, const double *s) {
  const double dx = __dsub_rn(x, s[0]), dy = __dsub_rn(y, s[1]), dz = __dsub_rn(z, s[2]);
  double d2 = __dmul_rn(dx, dx);
  d2 = __dadd_rn(d2, __dmul_rn(dy, dy));
  d2 = __dadd_rn(d2, __dmul_rn(dz, dz));
  return d2 <= __dmul_rn(s[3], s[3]);
}

// (Q - P) x (p - P) in the xy-plane: the side of p relative to the line P -> Q
__device__ __forceinline__ double edge_fn(const double *P, const double *Q, double x, double y) {
  return __dsub_rn(__dmul_rn(__dsub_rn(Q[0], P[0]), __dsub_rn(y, P[1])),
                   __dmul_rn(__dsub_rn(Q[1], P[1]), __dsub_rn(x, P[0])));
}

// inside the infinite prism (axis along z) over the triangle A B C, edges included
__device__ __forceinline__ bool in_prism(const double *A, const double *B, const double *C,
                                         double x, double y) {
  const double o = edge_fn(A, B, C[0], C[1]);
  const double e1 = edge_fn(A, B, x, y), e2 = edge_fn(B, C, x, y), e3 = edge_fn(C, A, x, y);
  return o > 0 ? (e1 >= 0 && e2 >= 0 && e3 >= 0) : (e1 <= 0 && e2 <= 0 && e3 <= 0);
}

}  // namespace geom
