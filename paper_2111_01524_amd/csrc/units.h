// The geometric tests and the per-unit rule of the flux truncation, shared by
// the kernels and by host builds of the same arithmetic (the operation counter
// of the measurements).  Every function here is plain FP64 arithmetic on its
// arguments, so the device and a host build compute the same values.
#pragma once
#include "clip.h"

namespace gvof {

__host__ __device__ inline int popc32(unsigned x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __popc(x);
#else
  return __builtin_popcount(x);
#endif
}

__host__ __device__ inline bool box_overlap(d3 alo, d3 ahi, d3 blo, d3 bhi) {
  return alo.x < bhi.x && blo.x < ahi.x && alo.y < bhi.y && blo.y < ahi.y && alo.z < bhi.z && blo.z < ahi.z;
}

// Flux tets of a face of I vertices: 3I (FMFPA), 5I (EMFPA), 3I-2 (NMFPA).
__host__ __device__ inline int flux_tet_count(int method, int I) {
  return method == kEMFPA ? 5 * I : (method == kNMFPA ? 3 * I - 2 : 3 * I);
}

// Flux tet t of the polyhedron (the fourth point is the face centre c), for
// edge i (j = i+1):
//   FMFPA kind 0 (x_j, x_i, b_j), 1 (x_i, b_i, b_j), 2 (a, b_j, b_i);
//   EMFPA kind 0 (x_j, x_i, m_i), 1 (x_i, b_i, m_i), 2 (b_i, b_j, m_i),
//         3 (b_j, x_j, m_i), 4 (a, b_j, b_i)
//   (the lateral quad x_j, x_i, b_i, b_j as four triangles to its centre);
//   NMFPA t < 2I: kinds 0 and 1 of FMFPA for edge t/2; t = 2I + k - 1
//   (k = 1..I-2): (b_0, b_{k+1}, b_k), the planar back face fanned from b_0.
__host__ __device__ inline void flux_tet_points(int t, int I, int method, int& i1, int& i2, int& i3) {
  const bool em = method == kEMFPA;
  const int i3e = t / 3, i5e = t / 5;  // constant divisions, both cheap
  if (method == kNMFPA) {
    const int i = t >> 1, kind = t & 1, k = t - 2 * I + 1;
    const int j = (i + 1 == I) ? 0 : i + 1;
    const bool back = k >= 1;
    i1 = back ? I : (kind == 0 ? j : i);
    i2 = back ? I + k + 1 : (kind == 0 ? i : I + i);
    i3 = back ? I + k : I + j;
    return;
  }
  const int i = em ? i5e : i3e, kind = t - (em ? 5 : 3) * i;
  const int j = (i + 1 == I) ? 0 : i + 1;
  if (em) {
    const int mi = 2 * I + 2 + i;
    i1 = kind == 0 ? j : kind == 1 ? i : kind == 2 ? I + i : kind == 3 ? I + j : 2 * I;
    i2 = kind == 0 ? i : kind == 1 ? I + i : kind == 2 ? I + j : kind == 3 ? j : I + j;
    i3 = kind == 4 ? I + i : mi;
  } else {
    i1 = kind == 0 ? j : (kind == 1 ? i : 2 * I);
    i2 = kind == 0 ? i : (kind == 1 ? I + i : I + j);
    i3 = kind == 0 ? I + j : (kind == 1 ? I + j : I + i);
  }
}

// Pairs with a general cell: which of the cell's surface tetrahedra (sigma)
// can share volume with the flux tet T, and how that volume is clipped.
// Every path (the staged filters, the deferred and overflow kernels) applies
// the same rule, so each unit set, each unit's value and hence each pair's sum
// are the same whichever path computes them:
//  - a sigma counts when its box meets T's, it is not flat, T is not entirely
//    outside one of its face planes, and it is not entirely outside one face
//    plane of T (then only a plane is common to both);
//  - the unit's volume vol(T ∩ sigma ∩ H) is found by clipping one of the two
//    by the face planes of the other that cut it: sigma by T's when fewer of
//    T's planes cut sigma than sigma's cut T, else T by sigma's.
// Unit word: the mask of the cutting planes (bits 0-3), whether the first of
// them keeps three tetrahedra (kUnitWideBit, a hint for grouping units of like
// work), and whether sigma is the one clipped (kUnitFlipBit).  Tc holds T's
// inward face planes and sc[l] the distance of the cell's vertex mean (the
// apex of every sigma) from plane l; the planes of sigma are those of
// tet_container(cc, t0, t1, t2), the planes of T those of
// tet_container(T.p0, T.p1, T.p2, T.p3).
constexpr int kUnitWideBit = 4;
constexpr int kUnitFlipBit = 5;
__host__ __device__ inline unsigned wide_bit(double s0, double s1, double s2, double s3) {
  return (s0 > 0.0) + (s1 > 0.0) + (s2 > 0.0) + (s3 > 0.0) >= 2 ? 1u : 0u;
}
__host__ __device__ inline bool unit_rule(const Tet& T, d3 tlo, d3 thi, const TetCont& Tc, const double (&sc)[4], d3 cc, d3 t0,
                                 d3 t1, d3 t2, unsigned& word) {
  word = 0;
  if (!box_overlap(tlo, thi, vmin(vmin(cc, t0), vmin(t1, t2)), vmax(vmax(cc, t0), vmax(t1, t2))) ||
      det3f(t0 - cc, t1 - cc, t2 - cc) == 0.0)
    return false;
  const TetCont TC = tet_container(cc, t0, t1, t2);
  unsigned cm = 0, wa = 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {  // sigma's planes against T
    const Plane P = TC.plane(l);
    const double s0 = P.dist(T.p0), s1 = P.dist(T.p1), s2 = P.dist(T.p2), s3 = P.dist(T.p3);
    if (fmax(fmax(s0, s1), fmax(s2, s3)) <= 0.0) return false;
    if (fmin(fmin(s0, s1), fmin(s2, s3)) < 0.0) {
      if (cm == 0u) wa = wide_bit(s0, s1, s2, s3);
      cm |= 1u << l;
    }
  }
  unsigned rm = 0, wb = 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {  // T's planes against sigma
    const Plane P = Tc.plane(l);
    const double s0 = sc[l], s1 = P.dist(t0), s2 = P.dist(t1), s3 = P.dist(t2);
    if (fmax(fmax(s0, s1), fmax(s2, s3)) <= 0.0) return false;
    if (fmin(fmin(s0, s1), fmin(s2, s3)) < 0.0) {
      if (rm == 0u) wb = wide_bit(s0, s1, s2, s3);
      rm |= 1u << l;
    }
  }
  const bool flip = popc32(rm) < popc32(cm);
  word = flip ? (rm | (rm ? wb << kUnitWideBit : 0u) | (1u << kUnitFlipBit)) : (cm | (cm ? wa << kUnitWideBit : 0u));
  return true;
}
// The unit's value as its word says: the clipped tet X, the other's planes C.
__host__ __device__ inline double unit_clip_value_setup(const Tet& T, d3 cc, d3 t0, d3 t1, d3 t2, unsigned word, Tet& X,
                                               TetCont& C) {
  const bool flip = (word >> kUnitFlipBit) & 1u;
  const Tet Sg{cc, t0, t1, t2};
  X = flip ? Sg : T;
  const Tet Y = flip ? T : Sg;
  C = tet_container(Y.p0, Y.p1, Y.p2, Y.p3);
  return 0.0;
}
// Distances of the cell's vertex mean from T's face planes.
__host__ __device__ inline void apex_dists(const TetCont& Tc, d3 cc, double (&sc)[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) sc[l] = Tc.plane(l).dist(cc);
}
// Cut mask of a tetrahedron with bounding box [tlo, thi] against box cell B,
// for a tetrahedron whose box meets B's (so it lies entirely outside no box
// plane): plane 2a (x_a >= lo_a) cuts it when a vertex has x_a < lo_a, plane
// 2a+1 (x_a <= hi_a) when a vertex has x_a > hi_a.  A box plane's distance
// is one rounded difference of two coordinates, whose sign is that of the
// exact difference, so this is cut_mask's result bit for bit.
__host__ __device__ inline unsigned box_cut_mask(d3 tlo, d3 thi, const BoxCont& B) {
  return (tlo.x < B.lo.x ? 1u : 0u) | (thi.x > B.hi.x ? 2u : 0u) | (tlo.y < B.lo.y ? 4u : 0u) |
         (thi.y > B.hi.y ? 8u : 0u) | (tlo.z < B.lo.z ? 16u : 0u) | (thi.z > B.hi.z ? 32u : 0u);
}


}  // namespace gvof
