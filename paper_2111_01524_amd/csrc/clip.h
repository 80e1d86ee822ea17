// Exact volume of a tetrahedron clipped by a convex container (an axis-aligned
// box or another tetrahedron) and optionally by one more half-space.
//
// The container's planes are applied by splitting: a tetrahedron cut by a
// plane keeps one tetrahedron (one vertex on the kept side), three (three
// vertices kept: a truncated prism) or three (two kept: a wedge).  Only the
// planes that cut the original tetrahedron are visited, depth first, with an
// explicit stack.  The last half-space is not split at all: every leaf adds
// its closed-form kept fraction (halfspace_fraction).
#pragma once
#include "gvof_dev.h"

namespace gvof {

// A plane as the affine function n.x + d (kept side >= 0).
struct Plane {
  d3 n;
  double d;
  __host__ __device__ inline double dist(d3 p) const { return dotf(n, p) + d; }
};

// Plane l of a container is picked with 0/1 weights, not with a chain of
// selects (which the compiler turns into a dynamically indexed private array,
// i.e. scratch memory).  With one weight 1 and the others 0 every sum below
// is exact, so the distances are those of the plain formulas bit for bit:
// for the box, x_a - lo_a and hi_a - x_a.
struct BoxCont {
  d3 lo, hi;
  static constexpr int np = 6;
  // plane l: axis l/2, l even -> x_a - lo_a >= 0, l odd -> hi_a - x_a >= 0
  __host__ __device__ inline Plane plane(int l) const {
    const int a = l >> 1;
    const bool up = (l & 1) != 0;
    const double ex = a == 0 ? 1.0 : 0.0, ey = a == 1 ? 1.0 : 0.0, ez = a == 2 ? 1.0 : 0.0;
    const double sg = up ? -1.0 : 1.0;
    const double blo = fma(ez, lo.z, fma(ey, lo.y, ex * lo.x)), bhi = fma(ez, hi.z, fma(ey, hi.y, ex * hi.x));
    return Plane{mk3(sg * ex, sg * ey, sg * ez), up ? bhi : -blo};
  }
  __host__ __device__ inline double dist(int l, d3 p) const { return plane(l).dist(p); }
};

struct TetCont {
  d3 n0, n1, n2, n3;
  double d0, d1, d2, d3_;
  static constexpr int np = 4;
  __host__ __device__ inline Plane plane(int l) const {
    const double w0 = l == 0 ? 1.0 : 0.0, w1 = l == 1 ? 1.0 : 0.0, w2 = l == 2 ? 1.0 : 0.0, w3 = l == 3 ? 1.0 : 0.0;
    d3 n = mk3(fma(w3, n3.x, fma(w2, n2.x, fma(w1, n1.x, w0 * n0.x))),
               fma(w3, n3.y, fma(w2, n2.y, fma(w1, n1.y, w0 * n0.y))),
               fma(w3, n3.z, fma(w2, n2.z, fma(w1, n1.z, w0 * n0.z))));
    double d = fma(w3, d3_, fma(w2, d2, fma(w1, d1, w0 * d0)));
    return Plane{n, d};
  }
  __host__ __device__ inline double dist(int l, d3 p) const { return plane(l).dist(p); }
};

// Inward half-spaces of the tetrahedron (a, b, c, d) as a point set.
__host__ __device__ inline TetCont tet_container(d3 a, d3 b, d3 c, d3 d) {
  if (det3f(b - a, c - a, d - a) < 0.0) {
    d3 t = c;
    c = d;
    d = t;
  }
  // outward faces (a,c,b), (a,b,d), (a,d,c), (b,c,d); inward normal = -(q-p)x(r-p)
  TetCont C;
  d3 N;
  N = crossf(c - a, b - a);
  C.n0 = mk3(-N.x, -N.y, -N.z);
  C.d0 = dotf(N, a);
  N = crossf(b - a, d - a);
  C.n1 = mk3(-N.x, -N.y, -N.z);
  C.d1 = dotf(N, a);
  N = crossf(d - a, c - a);
  C.n2 = mk3(-N.x, -N.y, -N.z);
  C.d2 = dotf(N, a);
  N = crossf(c - b, d - b);
  C.n3 = mk3(-N.x, -N.y, -N.z);
  C.d3_ = dotf(N, b);
  return C;
}

__host__ __device__ inline d3 cut_pt(d3 pin, double sin_, d3 pout, double sout) {
  double t = sin_ / (sin_ - sout);
  return axpy(t, pout - pin, pin);
}

// v unchanged, as a value the compiler cannot trace back to a load: a select
// between two such values stays a register select (a select between two
// loads is otherwise rewritten as a load from a selected address, which keeps
// the operands in scratch memory).
__host__ __device__ inline double opaque(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(v));
#endif
  return v;
}
__host__ __device__ inline int opaque(int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(v));
#endif
  return v;
}

// Orders (sa, pa), (sb, pb) so that sa >= sb (a swap: the values are unchanged).
__host__ __device__ inline void cs_pt(double& sa, d3& pa, double& sb, d3& pb) {
  const double s0 = opaque(sa), s1 = opaque(sb);
  const bool sw = s1 > s0;
  sa = sw ? s1 : s0;
  sb = sw ? s0 : s1;
  const double ax = opaque(pa.x), ay = opaque(pa.y), az = opaque(pa.z);
  const double bx = opaque(pb.x), by = opaque(pb.y), bz = opaque(pb.z);
  pa = mk3(sw ? bx : ax, sw ? by : ay, sw ? bz : az);
  pb = mk3(sw ? ax : bx, sw ? ay : by, sw ? az : bz);
}

struct Leaf {
  bool useH;
  d3 hn;
  double hd;
  __host__ __device__ inline double operator()(const Tet& t) const {
    double v = fabs(tet6(t)) * (1.0 / 6.0);
    if (!useH) return v;
    return v * halfspace_fraction(dotf(hn, t.p0) + hd, dotf(hn, t.p1) + hd, dotf(hn, t.p2) + hd,
                                  dotf(hn, t.p3) + hd);
  }
};

constexpr int kClipStack = 16;

// vol(T ∩ container ∩ {hn.x + hd >= 0 if useH}).  Returns -1 on stack overflow
// (cannot happen for <= 7 planes: depth-first keeps at most 2 siblings per level).
template <class Cont>
__host__ __device__ double clip_volume(const Tet& T, const Cont& C, const Leaf& leaf) {
  unsigned cut = 0;
  for (int l = 0; l < Cont::np; ++l) {
    double s0 = C.dist(l, T.p0), s1 = C.dist(l, T.p1), s2 = C.dist(l, T.p2), s3 = C.dist(l, T.p3);
    double mx = fmax(fmax(s0, s1), fmax(s2, s3)), mn = fmin(fmin(s0, s1), fmin(s2, s3));
    if (mx <= 0.0) return 0.0;
    if (mn < 0.0) cut |= 1u << l;
  }
  if (cut == 0) return leaf(T);
  Tet stk[kClipStack];
  unsigned char lvl[kClipStack];
  int sp = 1;
  stk[0] = T;
  lvl[0] = 0;
  double acc = 0.0;
  while (sp > 0) {
    --sp;
    Tet t = stk[sp];
    int l = lvl[sp];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    bool dropped = false;
    for (; l < Cont::np; ++l) {
      if (!((cut >> l) & 1u)) continue;
      s0 = C.dist(l, t.p0);
      s1 = C.dist(l, t.p1);
      s2 = C.dist(l, t.p2);
      s3 = C.dist(l, t.p3);
      double mx = fmax(fmax(s0, s1), fmax(s2, s3)), mn = fmin(fmin(s0, s1), fmin(s2, s3));
      if (mx <= 0.0) {
        dropped = true;
        break;
      }
      if (mn < 0.0) break;
    }
    if (dropped) continue;
    if (l >= Cont::np) {
      acc += leaf(t);
      continue;
    }
    // split t by plane l, keep s >= 0; vertices sorted by s, descending
    d3 a = t.p0, b = t.p1, c = t.p2, d = t.p3;
    double sa = s0, sb = s1, sc = s2, sd = s3;
    cs_pt(sa, a, sb, b);
    cs_pt(sc, c, sd, d);
    cs_pt(sa, a, sc, c);
    cs_pt(sb, b, sd, d);
    cs_pt(sb, b, sc, c);
    unsigned char nl = (unsigned char)(l + 1);
    if (sp + 3 > kClipStack) return -1.0;
    if (sb <= 0.0) {  // only a kept
      stk[sp] = Tet{a, cut_pt(a, sa, b, sb), cut_pt(a, sa, c, sc), cut_pt(a, sa, d, sd)};
      lvl[sp++] = nl;
    } else if (sc >= 0.0) {  // a, b, c kept, d dropped: truncated prism
      d3 pa = cut_pt(a, sa, d, sd), pb = cut_pt(b, sb, d, sd), pc = cut_pt(c, sc, d, sd);
      stk[sp] = Tet{a, b, c, pa};
      lvl[sp++] = nl;
      stk[sp] = Tet{b, c, pa, pb};
      lvl[sp++] = nl;
      stk[sp] = Tet{c, pa, pb, pc};
      lvl[sp++] = nl;
    } else {  // a, b kept, c, d dropped: wedge (a, P1, P2 | b, P3, P4)
      d3 P1 = cut_pt(a, sa, c, sc), P2 = cut_pt(a, sa, d, sd), P3 = cut_pt(b, sb, c, sc),
         P4 = cut_pt(b, sb, d, sd);
      stk[sp] = Tet{a, P1, P2, b};
      lvl[sp++] = nl;
      stk[sp] = Tet{P1, P2, b, P4};
      lvl[sp++] = nl;
      stk[sp] = Tet{P1, b, P4, P3};
      lvl[sp++] = nl;
    }
  }
  return acc;
}

// One split of a tetrahedron by an affine function with vertex values s
// (kept side s >= 0), with its children generated on demand so that a chain
// of splits stays in registers.
struct Split {
  d3 a, b, c, d;
  double sa, sb, sc, sd;
  d3 q0, q1, q2, q3;  // the cut points the children use, each computed once
  int kind;  // 0 nothing kept, 1 kept whole, 2 one vertex kept, 3 three kept (prism), 4 two kept (wedge)
  __host__ __device__ inline Split(const Tet& t, double s0, double s1, double s2, double s3) {
    a = t.p0; b = t.p1; c = t.p2; d = t.p3;
    sa = s0; sb = s1; sc = s2; sd = s3;
    double mx = fmax(fmax(s0, s1), fmax(s2, s3)), mn = fmin(fmin(s0, s1), fmin(s2, s3));
    if (mx <= 0.0) kind = 0;
    else if (mn >= 0.0) kind = 1;
    else {
      cs_pt(sa, a, sb, b);
      cs_pt(sc, c, sd, d);
      cs_pt(sa, a, sc, c);
      cs_pt(sb, b, sd, d);
      cs_pt(sb, b, sc, c);
      kind = (sb <= 0.0) ? 2 : ((sc >= 0.0) ? 3 : 4);
    }
    // edges cut: kind 2 ab ac ad, kind 3 ad bd cd, kind 4 ac ad bd bc
    const bool k2 = kind == 2, k3 = kind == 3;
    q0 = cut_pt(a, sa, k2 ? b : (k3 ? d : c), k2 ? sb : (k3 ? sd : sc));
    q1 = cut_pt(k3 ? b : a, k3 ? sb : sa, k2 ? c : d, k2 ? sc : sd);
    q2 = cut_pt(k2 ? a : (k3 ? c : b), k2 ? sa : (k3 ? sc : sb), d, sd);
    q3 = cut_pt(b, sb, c, sc);
  }
  __host__ __device__ inline int count() const { return kind == 0 ? 0 : (kind <= 2 ? 1 : 3); }
  // children by constant index (a runtime index makes the compiler keep the
  // three children in an indexed private array)
  __host__ __device__ inline Tet child0() const {
    const bool k1 = kind == 1, k2 = kind == 2, k3 = kind == 3;
    return Tet{a, (k1 || k3) ? b : q0, (k1 || k3) ? c : q1, k1 ? d : (k2 ? q2 : (k3 ? q0 : b))};
  }
  __host__ __device__ inline Tet child1() const {
    const bool k3 = kind == 3;
    return Tet{k3 ? b : q0, k3 ? c : q1, k3 ? q0 : b, k3 ? q1 : q2};
  }
  __host__ __device__ inline Tet child2() const {
    const bool k3 = kind == 3;
    return Tet{k3 ? c : q0, k3 ? q0 : b, k3 ? q1 : q2, k3 ? q2 : q3};
  }
  __host__ __device__ inline Tet child(int i) const { return i == 0 ? child0() : (i == 1 ? child1() : child2()); }
};

// Clip by one to four planes known to cut the original tetrahedron, in
// registers: the children of each split are visited in order 0, 1, 2 and
// summed in that order.
__host__ __device__ inline Split split_by(const Tet& t, const Plane& P) {
  return Split(t, P.dist(t.p0), P.dist(t.p1), P.dist(t.p2), P.dist(t.p3));
}
__host__ __device__ inline double clip1(const Tet& t, const Plane& P, const Leaf& leaf) {
  Split sp = split_by(t, P);
  const int n = sp.count();
  double acc = 0.0;
  if (n > 0) acc += leaf(sp.child0());
  if (n > 1) acc += leaf(sp.child1());
  if (n > 2) acc += leaf(sp.child2());
  return acc;
}
__host__ __device__ inline double clip2(const Tet& t, const Plane& P1, const Plane& P2, const Leaf& leaf) {
  Split sp = split_by(t, P1);
  const int n = sp.count();
  double acc = 0.0;
  if (n > 0) acc += clip1(sp.child0(), P2, leaf);
  if (n > 1) acc += clip1(sp.child1(), P2, leaf);
  if (n > 2) acc += clip1(sp.child2(), P2, leaf);
  return acc;
}
__host__ __device__ inline double clip3(const Tet& t, const Plane& P1, const Plane& P2, const Plane& P3,
                                         const Leaf& leaf) {
  Split sp = split_by(t, P1);
  const int n = sp.count();
  double acc = 0.0;
  if (n > 0) acc += clip2(sp.child0(), P2, P3, leaf);
  if (n > 1) acc += clip2(sp.child1(), P2, P3, leaf);
  if (n > 2) acc += clip2(sp.child2(), P2, P3, leaf);
  return acc;
}
// Compact forms for the rarely run deferred kernels: each level loops over
// the children instead of expanding them, which keeps those kernels small.
// The values and the order of the sums are those of the expanded forms.
__host__ __device__ __attribute__((always_inline)) inline double clip2c(const Tet& t, const Plane& P1,
                                                                        const Plane& P2, const Leaf& leaf) {
  Split sp = split_by(t, P1);
  const int n = sp.count();
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += clip1(sp.child(i), P2, leaf);
  return acc;
}
__host__ __device__ __attribute__((always_inline)) inline double clip3c(const Tet& t, const Plane& P1,
                                                                        const Plane& P2, const Plane& P3,
                                                                        const Leaf& leaf) {
  Split sp = split_by(t, P1);
  const int n = sp.count();
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += clip2c(sp.child(i), P2, P3, leaf);
  return acc;
}
__host__ __device__ __attribute__((always_inline)) inline double clip4c(const Tet& t, const Plane& P1,
                                                                        const Plane& P2, const Plane& P3,
                                                                        const Plane& P4, const Leaf& leaf) {
  Split sp = split_by(t, P1);
  const int n = sp.count();
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += clip3c(sp.child(i), P2, P3, P4, leaf);
  return acc;
}

// Up to four cutting planes of any container with the looping forms (-1
// beyond): the deferred kernels' clip.
template <class Cont>
__host__ __device__ __attribute__((always_inline)) inline double clip_masked_compact(const Tet& T, const Cont& C,
                                                                                     unsigned cut,
                                                                                     const Leaf& leaf) {
  Plane P[4] = {};
  int n = 0;
  unsigned rest = cut;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (rest) {
      int l = __builtin_ctz(rest);
      rest &= rest - 1u;
      const Plane pl = C.plane(l);
      P[0] = q == 0 ? pl : P[0];
      P[1] = q == 1 ? pl : P[1];
      P[2] = q == 2 ? pl : P[2];
      P[3] = q == 3 ? pl : P[3];
      ++n;
    }
  }
  if (rest) return -1.0;
  if (n == 0) return leaf(T);
  if (n == 1) return clip1(T, P[0], leaf);
  if (n == 2) return clip2c(T, P[0], P[1], leaf);
  if (n == 3) return clip3c(T, P[0], P[1], P[2], leaf);
  return clip4c(T, P[0], P[1], P[2], P[3], leaf);
}

// Cut mask of T against the container (bit l: plane l cuts T); returns false
// when T lies entirely outside one plane.
template <class Cont>
__host__ __device__ inline bool cut_mask(const Tet& T, const Cont& C, unsigned& cut) {
  cut = 0;
  for (int l = 0; l < Cont::np; ++l) {
    double s0 = C.dist(l, T.p0), s1 = C.dist(l, T.p1), s2 = C.dist(l, T.p2), s3 = C.dist(l, T.p3);
    double mx = fmax(fmax(s0, s1), fmax(s2, s3)), mn = fmin(fmin(s0, s1), fmin(s2, s3));
    if (mx <= 0.0) return false;
    if (mn < 0.0) cut |= 1u << l;
  }
  return true;
}

// vol(T ∩ container ∩ leaf half-space) for a precomputed cut mask with at
// most kMaxRegCuts cutting planes, in registers.  On the deformation workload
// over 99.9% of box pairs are cut by at most two box planes; callers send the
// rest to clip_volume (explicit stack) in a separate kernel.
constexpr int kMaxRegCuts = 2;
__host__ __device__ inline int cut_count(unsigned cut) {
  int n = 0;
  for (int l = 0; l < 6; ++l) n += (cut >> l) & 1u;
  return n;
}
template <class Cont>
__host__ __device__ __attribute__((always_inline)) inline double clip_masked(const Tet& T, const Cont& C, unsigned cut,
                                                                             const Leaf& leaf) {
  if (cut == 0) return leaf(T);
  int l1 = __builtin_ctz(cut);
  unsigned rest = cut & (cut - 1u);
  if (rest == 0) return clip1(T, C.plane(l1), leaf);
  return clip2(T, C.plane(l1), C.plane((int)__builtin_ctz(rest)), leaf);
}

// The same for a tetrahedron container: at most four cutting planes, all in
// registers (MAXC limits the depth compiled in; deeper masks return -1).
// COMPACT selects the looping forms (same values; small code for the rarely
// run deferred kernels).
template <int MAXC = 4, bool COMPACT = true>
__host__ __device__ __attribute__((always_inline)) inline double clip_masked_tet(const Tet& T, const TetCont& C,
                                                                                 unsigned cut, const Leaf& leaf) {
  int l[4] = {0, 0, 0, 0};
  int n = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if ((cut >> q) & 1u) {
      l[0] = n == 0 ? q : l[0];
      l[1] = n == 1 ? q : l[1];
      l[2] = n == 2 ? q : l[2];
      l[3] = n == 3 ? q : l[3];
      ++n;
    }
  }
  if (n == 0) return leaf(T);
  if (n == 1) return clip1(T, C.plane(l[0]), leaf);
  if (n == 2)
    return COMPACT ? clip2c(T, C.plane(l[0]), C.plane(l[1]), leaf) : clip2(T, C.plane(l[0]), C.plane(l[1]), leaf);
  if (MAXC >= 3 && n == 3)
    return COMPACT ? clip3c(T, C.plane(l[0]), C.plane(l[1]), C.plane(l[2]), leaf)
                   : clip3(T, C.plane(l[0]), C.plane(l[1]), C.plane(l[2]), leaf);
  if (MAXC >= 4) return clip4c(T, C.plane(l[0]), C.plane(l[1]), C.plane(l[2]), C.plane(l[3]), leaf);
  return -1.0;
}

// Volume of an axis-aligned box cut by {n.x >= s}: six Kuhn tetrahedra along
// the lo-hi diagonal, each V/6, closed form per tetrahedron.  lev[i] = n.corner_i
// with corner i = (i&1 ? hi.x : lo.x, i&2 ? hi.y : lo.y, i&4 ? hi.z : lo.z).
__host__ __device__ inline double box_level_volume(const double* lev, double V, double s) {
  double l0 = lev[0] - s, l7 = lev[7] - s;
  double l1 = lev[1] - s, l2 = lev[2] - s, l4 = lev[4] - s;
  double l3 = lev[3] - s, l5 = lev[5] - s, l6 = lev[6] - s;
  // paths 0 -> (1 | 2 | 4) -> (3 | 5 | 6) -> 7
  double f = halfspace_fraction(l0, l1, l3, l7) + halfspace_fraction(l0, l1, l5, l7) +
             halfspace_fraction(l0, l2, l3, l7) + halfspace_fraction(l0, l2, l6, l7) +
             halfspace_fraction(l0, l4, l5, l7) + halfspace_fraction(l0, l4, l6, l7);
  return V * (1.0 / 6.0) * f;
}

__host__ __device__ inline Tet kuhn_tet(d3 lo, d3 hi, int k) {
  // k: 0 x,y ; 1 x,z ; 2 y,x ; 3 y,z ; 4 z,x ; 5 z,y (first two axes of the path)
  int a1 = k >> 1;
  int a2 = (k == 0) ? 1 : (k == 1) ? 2 : (k == 2) ? 0 : (k == 3) ? 2 : (k == 4) ? 0 : 1;
  d3 p1 = lo, p2;
  if (a1 == 0) p1.x = hi.x;
  else if (a1 == 1) p1.y = hi.y;
  else p1.z = hi.z;
  p2 = p1;
  if (a2 == 0) p2.x = hi.x;
  else if (a2 == 1) p2.y = hi.y;
  else p2.z = hi.z;
  return Tet{lo, p1, p2, hi};
}

}  // namespace gvof
