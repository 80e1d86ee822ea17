// gVOF oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of the unsplit geometric VOF step of
// Lopez & Hernandez, "gVOF: An open-source package for unsplit geometric
// volume of fluid methods on arbitrary grids" (arXiv 2111.01524):
//   grid geometry (Sec. "Grid construction"), grid tagging (Sec. "Grid
//   tagging"), cut-off and PLIC (Sec. "Interface reconstruction", Eq.
//   plic-eq), LSGIR normals (Sec. LSGIR, Eqs. lsgir1, lsgir2, lsgir-beta)
//   optionally refined by LSFIR (Sec. "Least squares fit interface
//   reconstruction"),
//   the plane constant enforcing the cell's volume fraction, face flux
//   volumes (Eq. a-donacion), FMFPA flux polyhedra (Sec. "Face-matched flux
//   polyhedron"), EMFPA ones (Sec. "Edge-matched flux polyhedron") or NMFPA
//   ones (Sec. "Non-matched flux polyhedron"), chosen per mesh, their
//   truncation by the PLIC half-spaces of the cells they
//   overlap (Sec. "Fluid advected through cell faces") and the volume fraction
//   update with clamp (Eq. fnext), plus the refinement initialisation (Sec.
//   "Fluid volume fraction initialization").
//
// Only the test-suite, the smoke check and the CPU baseline of the benchmark
// load this library.  It shares no source with the HIP library.  Geometry is
// done with the most direct methods available: convex polyhedra as face
// lists clipped one plane at a time (Sutherland-Hodgman on every face plus a
// cap polygon made of the cut points sorted by angle), volumes by fanning
// every face from a reference point.  Non-convex cells and flux polyhedra are
// signed sums of tetrahedra (winding-number integration), which is exact for
// self-intersecting surfaces.
//
// Readings of points the paper leaves open are listed where they are used;
// every one of them is shared by the HIP library's design notes.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_COUNT_FLOPS
#include "counted_real.h"
long long g_orc_flops = 0;
using real = CountedReal;
#else
using real = double;
static inline double to_double(double a) { return a; }
#endif
using std::atan2;
using std::fabs;
using std::pow;
using std::sqrt;

namespace {

struct V3 {
  real x, y, z;
};
inline V3 mk(real x, real y, real z) { return V3{x, y, z}; }
inline V3 operator+(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
inline V3 operator-(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
inline V3 operator*(real s, V3 a) { return mk(s * a.x, s * a.y, s * a.z); }
// Fixed evaluation order (x, then y, then z) so that branch-deciding values are
// reproducible bit for bit by any implementation that keeps the same order.
inline real dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
inline real det3(V3 a, V3 b, V3 c) { return dot(a, cross(b, c)); }

// --------------------------------------------------------------------------
// Convex polyhedra as face lists.
// --------------------------------------------------------------------------
struct Poly {
  std::vector<std::vector<V3>> faces;  // each face counter-clockwise seen from outside
};

// A tetrahedron as a point set, faces oriented outward.
Poly tet_poly(V3 a, V3 b, V3 c, V3 d) {
  if (det3(b - a, c - a, d - a) < real(0.0)) std::swap(c, d);
  Poly P;
  P.faces = {{a, c, b}, {a, b, d}, {a, d, c}, {b, c, d}};
  return P;
}

Poly box_poly(V3 lo, V3 hi) {
  auto p = [&](int i, int j, int k) { return mk(i ? hi.x : lo.x, j ? hi.y : lo.y, k ? hi.z : lo.z); };
  Poly P;
  P.faces = {{p(0, 0, 0), p(0, 0, 1), p(0, 1, 1), p(0, 1, 0)},   // -x
             {p(1, 0, 0), p(1, 1, 0), p(1, 1, 1), p(1, 0, 1)},   // +x
             {p(0, 0, 0), p(1, 0, 0), p(1, 0, 1), p(0, 0, 1)},   // -y
             {p(0, 1, 0), p(0, 1, 1), p(1, 1, 1), p(1, 1, 0)},   // +y
             {p(0, 0, 0), p(0, 1, 0), p(1, 1, 0), p(1, 0, 0)},   // -z
             {p(0, 0, 1), p(1, 0, 1), p(1, 1, 1), p(0, 1, 1)}};  // +z
  return P;
}

// Cut point on the edge from a kept vertex to a removed one, always computed
// from the kept side so both faces sharing the edge get the same bits.
inline V3 cut_point(V3 pin, real sin_, V3 pout, real sout) {
  real t = sin_ / (sin_ - sout);
  return pin + t * (pout - pin);
}

// Signed distances within a few rounding errors of zero count as exactly on
// the plane: a face that lies on the plane in exact arithmetic then neither
// cuts off a sliver nor produces a degenerate cap (the rounding-level sliver
// it would remove has volume far below the parity tolerance).
real snap_tol(const Poly& P, V3 n, real d) {
  real scale = 0.0;
  for (auto& f : P.faces)
    for (auto& p : f) scale = std::max(scale, std::max(fabs(p.x), std::max(fabs(p.y), fabs(p.z))));
  return real(4e-15) * (sqrt(dot(n, n)) * scale + fabs(d));
}

inline real sdist(V3 n, real d, V3 p, real tol) {
  real s = dot(n, p) + d;
  return fabs(s) <= tol ? real(0.0) : s;
}

// Keep the part of P where n.x + d >= 0.
void clip(Poly& P, V3 n, real d) {
  real tol = snap_tol(P, n, d);
  bool any_in = false, any_out = false;
  for (auto& f : P.faces)
    for (auto& p : f) {
      real s = sdist(n, d, p, tol);
      if (s > real(0.0)) any_in = true;
      if (s < real(0.0)) any_out = true;
    }
  if (!any_out) return;                  // plane does not cut
  if (!any_in) { P.faces.clear(); return; }  // nothing of positive volume left
  std::vector<std::vector<V3>> out;
  std::vector<V3> cap;
  for (auto& f : P.faces) {
    std::vector<V3> g;
    size_t k = f.size();
    for (size_t i = 0; i < k; ++i) {
      V3 a = f[i], b = f[(i + 1) % k];
      real sa = sdist(n, d, a, tol), sb = sdist(n, d, b, tol);
      bool ia = sa >= real(0.0), ib = sb >= real(0.0);
      if (ia) {
        g.push_back(a);
        if (sa == real(0.0)) cap.push_back(a);
      }
      if (ia && !ib) { V3 c = cut_point(a, sa, b, sb); g.push_back(c); cap.push_back(c); }
      if (!ia && ib) { V3 c = cut_point(b, sb, a, sa); g.push_back(c); cap.push_back(c); }
    }
    if (g.size() >= 3) out.push_back(g);
  }
  if (cap.size() >= 3) {
    // cap polygon: its outward normal is -n; order the points by angle about their mean
    V3 cen = mk(0.0, 0.0, 0.0);
    for (auto& p : cap) cen = cen + p;
    cen = (real(1.0) / real(double(cap.size()))) * cen;
    V3 N = mk(-n.x, -n.y, -n.z);
    V3 ax = (fabs(N.x) <= fabs(N.y) && fabs(N.x) <= fabs(N.z)) ? mk(1.0, 0.0, 0.0)
            : (fabs(N.y) <= fabs(N.z) ? mk(0.0, 1.0, 0.0) : mk(0.0, 0.0, 1.0));
    V3 e1 = cross(N, ax);
    V3 e2 = cross(N, e1);  // (e1, e2, N) right-handed up to scale
    std::vector<std::pair<double, V3>> ang;
    for (auto& p : cap) {
      V3 q = p - cen;
      ang.push_back({to_double(atan2(dot(q, e2), dot(q, e1))), p});
    }
    std::stable_sort(ang.begin(), ang.end(),
                     [](const std::pair<double, V3>& u, const std::pair<double, V3>& v) { return u.first < v.first; });
    std::vector<V3> g;
    for (auto& a : ang) g.push_back(a.second);
    out.push_back(g);
  }
  P.faces.swap(out);
}

real volume(const Poly& P) {
  if (P.faces.empty()) return real(0.0);
  V3 r = P.faces[0][0];
  real v = 0.0;
  for (auto& f : P.faces)
    for (size_t i = 1; i + 1 < f.size(); ++i) v = v + det3(f[0] - r, f[i] - r, f[i + 1] - r);
  return v / real(6.0);
}

struct Plane {
  V3 n;
  real d;  // half-space n.x + d >= 0
};

// The four inward half-spaces of a tetrahedron (a point set).
void tet_planes(V3 a, V3 b, V3 c, V3 d, Plane out[4]) {
  if (det3(b - a, c - a, d - a) < real(0.0)) std::swap(c, d);
  V3 f[4][3] = {{a, c, b}, {a, b, d}, {a, d, c}, {b, c, d}};
  for (int i = 0; i < 4; ++i) {
    V3 N = cross(f[i][1] - f[i][0], f[i][2] - f[i][0]);  // outward
    out[i].n = mk(-N.x, -N.y, -N.z);
    out[i].d = dot(N, f[i][0]);
  }
}

// --------------------------------------------------------------------------
// Mesh
// --------------------------------------------------------------------------
struct Tet {  // a cell's surface triangle fanned from the cell centre
  V3 p[4];
  real sign;
};

struct OMesh {
  int nv = 0, nf = 0, nc = 0;
  std::vector<V3> X;
  std::vector<int> fptr, fidx, owner, neigh;
  // topology
  std::vector<std::vector<std::pair<int, int>>> cf;  // cell -> (face, sigma) ascending face
  std::vector<std::vector<int>> cv;                  // cell -> distinct vertices ascending
  std::vector<std::vector<int>> vc;                  // vertex -> cells ascending
  std::vector<std::vector<int>> nb;                  // cell -> vertex-sharing cells (not itself) ascending
  // geometry
  std::vector<V3> S, fc, cc, bbmin, bbmax;
  V3 dom_lo, dom_hi;  // enclosing box of every vertex (of the whole domain)
  std::vector<real> V;
  std::vector<char> isbox;
  std::vector<std::vector<Tet>> tets;  // surface tets of every non-box cell
  int method = 0;                      // flux polyhedra: 0 FMFPA, 1 EMFPA, 2 NMFPA
  int recon = 0;                       // normals: 0 LSGIR, 1 LSFIR, 2 LLCIR, 3 ELCIR, 4 CLCIR
  int lsfir_outer = 4;                 // LSFIR outer iterations at most (the paper's tests: 4)
  double lsfir_tol = 1e-3;             // LSFIR: stop once no normal turns by this angle (rad) or more (1e-3)
  bool lsfir_cap = false;              // LSFIR weight floor at |d| = 0.05 h (not the paper's; opt-in)
};

// Surface triangles of cell c: triangle faces as they are, polygons fanned
// from their vertex mean; every triangle oriented outward of c.
void cell_triangles(const OMesh& M, int c, std::vector<std::array<V3, 3>>& tri) {
  tri.clear();
  for (auto& fs : M.cf[c]) {
    int f = fs.first, sg = fs.second;
    int b = M.fptr[f], k = M.fptr[f + 1] - b;
    if (k == 3) {
      V3 a0 = M.X[M.fidx[b]], a1 = M.X[M.fidx[b + 1]], a2 = M.X[M.fidx[b + 2]];
      if (sg > 0) tri.push_back({a0, a1, a2});
      else tri.push_back({a0, a2, a1});
    } else {
      for (int i = 0; i < k; ++i) {
        V3 a = M.X[M.fidx[b + i]], bb = M.X[M.fidx[b + (i + 1) % k]];
        if (sg > 0) tri.push_back({M.fc[f], a, bb});
        else tri.push_back({M.fc[f], bb, a});
      }
    }
  }
}

void build_mesh(OMesh& M) {
  int nv = M.nv, nf = M.nf, nc = M.nc;
  M.dom_lo = M.dom_hi = M.X[0];
  for (int v = 1; v < nv; ++v) {
    M.dom_lo = mk(std::min(M.dom_lo.x, M.X[v].x), std::min(M.dom_lo.y, M.X[v].y), std::min(M.dom_lo.z, M.X[v].z));
    M.dom_hi = mk(std::max(M.dom_hi.x, M.X[v].x), std::max(M.dom_hi.y, M.X[v].y), std::max(M.dom_hi.z, M.X[v].z));
  }
  M.cf.assign(nc, {});
  for (int f = 0; f < nf; ++f) {
    M.cf[M.owner[f]].push_back({f, +1});
    if (M.neigh[f] >= 0) M.cf[M.neigh[f]].push_back({f, -1});
  }
  M.cv.assign(nc, {});
  for (int c = 0; c < nc; ++c) {
    std::vector<int> vs;
    for (auto& fs : M.cf[c])
      for (int i = M.fptr[fs.first]; i < M.fptr[fs.first + 1]; ++i) vs.push_back(M.fidx[i]);
    std::sort(vs.begin(), vs.end());
    vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
    M.cv[c] = vs;
  }
  M.vc.assign(nv, {});
  for (int c = 0; c < nc; ++c)
    for (int v : M.cv[c]) M.vc[v].push_back(c);  // c ascending by construction
  M.nb.assign(nc, {});
  for (int c = 0; c < nc; ++c) {
    std::vector<int> ns;
    for (int v : M.cv[c])
      for (int k : M.vc[v])
        if (k != c) ns.push_back(k);
    std::sort(ns.begin(), ns.end());
    ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
    M.nb[c] = ns;
  }
  // face geometry: centre = vertex mean, area vector = half the sum of the
  // fan cross products about the centre (planar faces give the exact area).
  M.S.assign(nf, mk(0.0, 0.0, 0.0));
  M.fc.assign(nf, mk(0.0, 0.0, 0.0));
  for (int f = 0; f < nf; ++f) {
    int b = M.fptr[f], k = M.fptr[f + 1] - b;
    V3 s = mk(0.0, 0.0, 0.0);
    for (int i = 0; i < k; ++i) s = s + M.X[M.fidx[b + i]];
    real ik = real(double(k));
    V3 c = mk(s.x / ik, s.y / ik, s.z / ik);
    V3 A = mk(0.0, 0.0, 0.0);
    for (int i = 0; i < k; ++i) {
      V3 p = M.X[M.fidx[b + i]] - c, q = M.X[M.fidx[b + (i + 1) % k]] - c;
      A = A + cross(p, q);
    }
    M.fc[f] = c;
    M.S[f] = mk(real(0.5) * A.x, real(0.5) * A.y, real(0.5) * A.z);
  }
  // cell geometry: centre = mean of the distinct vertices (ascending id),
  // enclosing box, volume = signed tets from the centre over the surface.
  M.cc.assign(nc, mk(0.0, 0.0, 0.0));
  M.bbmin.assign(nc, mk(0.0, 0.0, 0.0));
  M.bbmax.assign(nc, mk(0.0, 0.0, 0.0));
  M.V.assign(nc, 0.0);
  M.isbox.assign(nc, 0);
  M.tets.assign(nc, {});
  std::vector<std::array<V3, 3>> tri;
  for (int c = 0; c < nc; ++c) {
    V3 s = mk(0.0, 0.0, 0.0), lo = M.X[M.cv[c][0]], hi = lo;
    for (int v : M.cv[c]) {
      V3 p = M.X[v];
      s = s + p;
      lo = mk(std::min(lo.x, p.x), std::min(lo.y, p.y), std::min(lo.z, p.z));
      hi = mk(std::max(hi.x, p.x), std::max(hi.y, p.y), std::max(hi.z, p.z));
    }
    real in = real(double(M.cv[c].size()));
    V3 cen = mk(s.x / in, s.y / in, s.z / in);
    M.cc[c] = cen;
    M.bbmin[c] = lo;
    M.bbmax[c] = hi;
    // box: six quadrilaterals, eight distinct vertices all at corners of the enclosing box
    bool box = M.cv[c].size() == 8 && M.cf[c].size() == 6;
    if (box) {
      int mask = 0;
      for (int v : M.cv[c]) {
        V3 p = M.X[v];
        bool okx = p.x == lo.x || p.x == hi.x, oky = p.y == lo.y || p.y == hi.y, okz = p.z == lo.z || p.z == hi.z;
        if (!(okx && oky && okz)) { box = false; break; }
        mask |= 1 << ((p.x == hi.x ? 1 : 0) + (p.y == hi.y ? 2 : 0) + (p.z == hi.z ? 4 : 0));
      }
      if (box && mask != 255) box = false;
      if (box && !(lo.x < hi.x && lo.y < hi.y && lo.z < hi.z)) box = false;
      for (auto& fs : M.cf[c])
        if (M.fptr[fs.first + 1] - M.fptr[fs.first] != 4) box = false;
    }
    M.isbox[c] = box ? 1 : 0;
    cell_triangles(M, c, tri);
    real vol = 0.0;
    for (auto& t : tri) {
      real d = det3(t[0] - cen, t[1] - cen, t[2] - cen);
      vol = vol + d;
      if (!box) M.tets[c].push_back(Tet{{cen, t[0], t[1], t[2]}, d > real(0.0) ? real(1.0) : real(-1.0)});
    }
    M.V[c] = vol / real(6.0);
  }
}

inline bool boxes_overlap(V3 alo, V3 ahi, V3 blo, V3 bhi) {
  return alo.x < bhi.x && blo.x < ahi.x && alo.y < bhi.y && blo.y < ahi.y && alo.z < bhi.z && blo.z < ahi.z;
}

void tet_bbox(const V3* p, V3& lo, V3& hi) {
  lo = hi = p[0];
  for (int i = 1; i < 4; ++i) {
    lo = mk(std::min(lo.x, p[i].x), std::min(lo.y, p[i].y), std::min(lo.z, p[i].z));
    hi = mk(std::max(hi.x, p[i].x), std::max(hi.y, p[i].y), std::max(hi.z, p[i].z));
  }
}

// vol(tet T ∩ cell c [∩ {n.x + C >= 0}]).  For non-box cells this is the
// signed sum over the cell's surface tets (exact for non-convex cells).
real tet_cell_volume(const OMesh& M, const V3* T, int c, bool use_plane, V3 n, real C) {
  V3 tlo, thi;
  tet_bbox(T, tlo, thi);
  if (!boxes_overlap(tlo, thi, M.bbmin[c], M.bbmax[c])) return real(0.0);
  if (M.isbox[c]) {
    Poly P = tet_poly(T[0], T[1], T[2], T[3]);
    V3 lo = M.bbmin[c], hi = M.bbmax[c];
    clip(P, mk(1.0, 0.0, 0.0), -lo.x);
    clip(P, mk(-1.0, 0.0, 0.0), hi.x);
    clip(P, mk(0.0, 1.0, 0.0), -lo.y);
    clip(P, mk(0.0, -1.0, 0.0), hi.y);
    clip(P, mk(0.0, 0.0, 1.0), -lo.z);
    clip(P, mk(0.0, 0.0, -1.0), hi.z);
    if (use_plane) clip(P, n, C);
    return volume(P);
  }
  real acc = 0.0;
  for (const Tet& s : M.tets[c]) {
    V3 slo, shi;
    tet_bbox(s.p, slo, shi);
    if (!boxes_overlap(tlo, thi, slo, shi)) continue;
    Plane pl[4];
    tet_planes(s.p[0], s.p[1], s.p[2], s.p[3], pl);
    Poly P = tet_poly(T[0], T[1], T[2], T[3]);
    for (int i = 0; i < 4; ++i) clip(P, pl[i].n, pl[i].d);
    if (use_plane) clip(P, n, C);
    acc = acc + s.sign * volume(P);
  }
  return acc;
}

// vol(cell c ∩ {n.x >= s})
real cell_level_volume(const OMesh& M, int c, V3 n, real s) {
  if (M.isbox[c]) {
    Poly P = box_poly(M.bbmin[c], M.bbmax[c]);
    clip(P, n, -s);
    return volume(P);
  }
  real acc = 0.0;
  for (const Tet& t : M.tets[c]) {
    Poly P = tet_poly(t.p[0], t.p[1], t.p[2], t.p[3]);
    clip(P, n, -s);
    acc = acc + t.sign * volume(P);
  }
  return acc;
}

// --------------------------------------------------------------------------
// Grid tagging (Sec. "Grid tagging"): node value by inverse distance
// weighting (power 2 -- the paper names no power), then node, face and cell
// tags in {-1, 0, 1}.
// --------------------------------------------------------------------------
void node_values(const OMesh& M, const double* F, std::vector<real>& Fs) {
  Fs.assign(M.nv, 0.0);
#pragma omp parallel for schedule(static)
  for (int v = 0; v < M.nv; ++v) {
    real num = 0.0, den = 0.0;
    for (int c : M.vc[v]) {
      V3 d = M.X[v] - M.cc[c];
      real d2 = (d.x * d.x + d.y * d.y) + d.z * d.z;
      real w = real(1.0) / d2;
      num = num + w * real(F[c]);
      den = den + w;
    }
    Fs[v] = num / den;
  }
}

inline int8_t tag_of(real f, real eps) {
  if (f < eps) return -1;
  if (f > real(1.0) - eps) return 1;
  return 0;
}

void tags(const OMesh& M, const double* F, double eps, std::vector<real>& Fs, int8_t* tn, int8_t* tf, int8_t* tc) {
  node_values(M, F, Fs);
  for (int v = 0; v < M.nv; ++v) tn[v] = tag_of(Fs[v], eps);
  for (int f = 0; f < M.nf; ++f) {
    bool allm = true, allp = true;
    for (int i = M.fptr[f]; i < M.fptr[f + 1]; ++i) {
      int8_t t = tn[M.fidx[i]];
      if (t != -1) allm = false;
      if (t != 1) allp = false;
    }
    tf[f] = allm ? -1 : (allp ? 1 : 0);
  }
  for (int c = 0; c < M.nc; ++c) tc[c] = tag_of(real(F[c]), eps);
}

// --------------------------------------------------------------------------
// LSGIR (Sec. LSGIR): grad F = (A^T A)^{-1} A^T b with rows w_k (x_k - x)
// and w_k (F_k - F), w_k = |x - x_k|^{-beta}, over the cells sharing a
// vertex; n = grad F / |grad F|.  Normal equations solved by Gaussian
// elimination with partial pivoting.  Zero gradient -> n = (0,0,1).
// --------------------------------------------------------------------------
V3 lsgir_normal(const OMesh& M, const double* F, int c, double beta) {
  real A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, r[3] = {0, 0, 0};
  for (int k : M.nb[c]) {
    V3 d = M.cc[k] - M.cc[c];
    real dist = sqrt(dot(d, d));
    real w = pow(dist, real(-beta));
    real w2 = w * w;
    real df = real(F[k]) - real(F[c]);
    real dv[3] = {d.x, d.y, d.z};
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) A[i][j] = A[i][j] + w2 * dv[i] * dv[j];
      r[i] = r[i] + w2 * dv[i] * df;
    }
  }
  // Gaussian elimination with partial pivoting
  int p[3] = {0, 1, 2};
  for (int col = 0; col < 3; ++col) {
    int best = col;
    for (int i = col + 1; i < 3; ++i)
      if (fabs(A[p[i]][col]) > fabs(A[p[best]][col])) best = i;
    std::swap(p[col], p[best]);
    real piv = A[p[col]][col];
    if (piv == real(0.0)) return mk(0.0, 0.0, 1.0);
    for (int i = col + 1; i < 3; ++i) {
      real m = A[p[i]][col] / piv;
      for (int j = col; j < 3; ++j) A[p[i]][j] = A[p[i]][j] - m * A[p[col]][j];
      r[p[i]] = r[p[i]] - m * r[p[col]];
    }
  }
  real g[3];
  for (int i = 2; i >= 0; --i) {
    real s = r[p[i]];
    for (int j = i + 1; j < 3; ++j) s = s - A[p[i]][j] * g[j];
    g[i] = s / A[p[i]][i];
  }
  real nn = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
  if (nn == real(0.0)) return mk(0.0, 0.0, 1.0);
  real inv = real(1.0) / sqrt(nn);
  return mk(g[0] * inv, g[1] * inv, g[2] * inv);
}

// Plane constant: the unique C with vol(cell ∩ {n.x + C >= 0}) = F V, by
// bisection on a level between the extreme vertex levels.  The smaller of
// the fluid and empty volumes is matched: for F > 1/2 the empty part
// vol(cell ∩ {-n.x >= s}) = (1 - F) V (1 - F exact there), which defines the
// same plane but is evaluated with rounding relative to the small volume, so
// a nearly full cell's plane is as well determined as a nearly empty one's.
real plane_constant(const OMesh& M, int c, V3 n, double Fc) {
  const bool flip = Fc > 0.5;
  const V3 m = flip ? mk(-n.x, -n.y, -n.z) : n;
  real lo = dot(m, M.X[M.cv[c][0]]), hi = lo;
  for (int v : M.cv[c]) {
    real s = dot(m, M.X[v]);
    lo = std::min(lo, s);
    hi = std::max(hi, s);
  }
  real target = (flip ? real(1.0) - real(Fc) : real(Fc)) * M.V[c];
  for (int it = 0; it < 400; ++it) {
    real mid = real(0.5) * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (cell_level_volume(M, c, m, mid) > target) lo = mid;
    else hi = mid;
  }
  real s = real(0.5) * (lo + hi);
  return flip ? s : -s;  // fluid {n.x >= -s}, or the complement of {-n.x >= s}
}

// --------------------------------------------------------------------------
// LSFIR (Sec. "Least squares fit interface reconstruction").
// --------------------------------------------------------------------------

// Geometric centre of the PLIC polygon {n.x + C = 0} within cell c: the mean
// of its vertices, which are the cell's vertices lying on the plane and the
// crossing points of the cell's edges whose ends lie strictly on opposite
// sides.  Vertices in ascending order, then edges (each once, as ascending
// vertex pairs) in ascending order.  Returns the number of points (0: the
// plane misses the cell, the centre is then the cell centre).
int plic_centre(const OMesh& M, int c, V3 n, real C, V3& out) {
  std::vector<std::pair<int, int>> edges;
  for (auto& fs : M.cf[c]) {
    int f = fs.first, b = M.fptr[f], k = M.fptr[f + 1] - b;
    for (int i = 0; i < k; ++i) {
      int a = M.fidx[b + i], e = M.fidx[b + (i + 1) % k];
      edges.push_back({std::min(a, e), std::max(a, e)});
    }
  }
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  V3 sum = mk(0.0, 0.0, 0.0);
  int cnt = 0;
  for (int v : M.cv[c]) {
    if (dot(n, M.X[v]) + C == real(0.0)) {
      sum = sum + M.X[v];
      ++cnt;
    }
  }
  for (auto& e : edges) {
    V3 xa = M.X[e.first], xb = M.X[e.second];
    real sa = dot(n, xa) + C, sb = dot(n, xb) + C;
    if ((sa > real(0.0) && sb < real(0.0)) || (sa < real(0.0) && sb > real(0.0))) {
      real t = sa / (sa - sb);
      sum = sum + (xa + t * (xb - xa));
      ++cnt;
    }
  }
  if (cnt == 0) {
    out = M.cc[c];
    return 0;
  }
  real k = real(double(cnt));
  out = mk(sum.x / k, sum.y / k, sum.z / k);
  return cnt;
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (the textbook method): on return the diagonal of A holds the eigenvalues
// and the columns of V the eigenvectors.
void jacobi3(real A[3][3], real V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? real(1.0) : real(0.0);
  for (int sweep = 0; sweep < 64; ++sweep) {
    real off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    if (off == real(0.0)) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == real(0.0)) continue;
        real theta = (A[q][q] - A[p][p]) / (real(2.0) * A[p][q]);
        real t = real(1.0) / (fabs(theta) + sqrt(theta * theta + real(1.0)));
        if (theta < real(0.0)) t = -t;
        real cs = real(1.0) / sqrt(t * t + real(1.0)), sn = t * cs;
        // A <- R^T A R with the rotation in the (p, q) plane
        for (int k = 0; k < 3; ++k) {
          real akp = A[k][p], akq = A[k][q];
          A[k][p] = cs * akp - sn * akq;
          A[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < 3; ++k) {
          real apk = A[p][k], aqk = A[q][k];
          A[p][k] = cs * apk - sn * aqk;
          A[q][k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          real vkp = V[k][p], vkq = V[k][q];
          V[k][p] = cs * vkp - sn * vkq;
          V[k][q] = sn * vkp + cs * vkq;
        }
      }
    }
  }
}

// One least-squares fit: the unit normal of the plane through the PLIC centre
// x of cell c that minimises sum w_k (n.(x_k - x))^2 over the valid
// neighbours k (interfacial cells sharing a vertex with c whose normals
// differ from c's by less than 45 degrees), w_k = |x_k - x|^-2.5 (the
// section's weight; a neighbour whose centre coincides with x has no
// direction and is skipped): the eigenvector of the smallest eigenvalue of
// sum w_k d_k d_k^T, turned to agree with c's normal.  Keeps c's normal when
// fewer than two neighbours are valid or the smallest eigenvalue is not
// separated from the next.  With lsfir_cap (an option the paper does not
// have) the weight of a centre closer than 0.05 h is taken at |d| = 0.05 h
// (h: the largest extent of c's box).
V3 lsfir_fit(const OMesh& M, int c, const std::vector<V3>& nrm, const std::vector<V3>& xc, const int8_t* tc,
             int& nvalid) {
  const real cos45 = sqrt(real(0.5));
  V3 ext = M.bbmax[c] - M.bbmin[c];
  real hc = std::max(std::max(ext.x, ext.y), ext.z);
  real dmin2 = M.lsfir_cap ? (real(0.05) * hc) * (real(0.05) * hc) : real(0.0);
  real A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  nvalid = 0;
  for (int k : M.nb[c]) {
    if (tc[k] != 0) continue;
    if (!(dot(nrm[c], nrm[k]) > cos45)) continue;
    V3 d = xc[k] - xc[c];
    real dd = dot(d, d);
    if (dd == real(0.0)) continue;
    real dw = std::max(dd, dmin2);  // dd itself unless the floor is on
    real w = real(1.0) / (dw * sqrt(sqrt(dw)));  // |d|^-2.5
    real dv[3] = {d.x, d.y, d.z};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[i][j] = A[i][j] + w * dv[i] * dv[j];
    ++nvalid;
  }
  if (nvalid < 2) return nrm[c];
  real V[3][3];
  jacobi3(A, V);
  int i0 = 0, i1 = 1, i2 = 2;  // eigenvalues ascending
  if (A[i1][i1] < A[i0][i0]) std::swap(i0, i1);
  if (A[i2][i2] < A[i1][i1]) std::swap(i1, i2);
  if (A[i1][i1] < A[i0][i0]) std::swap(i0, i1);
  real l0 = A[i0][i0], l1 = A[i1][i1], l2 = A[i2][i2];
  if (!(l1 - l0 > real(1e-12) * l2)) return nrm[c];
  V3 e = mk(V[0][i0], V[1][i0], V[2][i0]);
  real en = sqrt(dot(e, e));
  e = mk(e.x / en, e.y / en, e.z / en);
  if (dot(e, nrm[c]) < real(0.0)) e = mk(-e.x, -e.y, -e.z);
  return e;
}


// --------------------------------------------------------------------------
// Isosurface-based reconstruction (Sec. "Isosurface based interface
// reconstruction": LLCIR, ELCIR, CLCIR).
// --------------------------------------------------------------------------

// The isosurface F* = 1/2 of cell c as one polygon.  A vertex is inside when
// F* >= 1/2.  Every cell edge whose ends differ crosses the isosurface at the
// linear-interpolation point (computed from the edge's lower vertex index,
// so both faces of the edge get the same point).  On each face, taken in
// the cell's outward orientation, the crossings go in pairs: a segment from
// the crossing where the walk enters the inside to the one where it leaves.
// The segments, chained end to start, form the polygon.  Returns false (no
// usable isosurface) when min F* < 1/2 < max F* fails, a face has more than
// two crossings, or the segments form more than one loop.  cyc: the points
// in loop order from the segment of the cell's first face that has one;
// cface: the face each polygon edge (cyc[i], cyc[i+1]) lies on.
bool iso_polygon(const OMesh& M, int c, const std::vector<real>& Fs, std::vector<V3>& cyc, std::vector<int>& cface) {
  cyc.clear();
  cface.clear();
  real fmin = Fs[M.cv[c][0]], fmax = fmin;
  for (int v : M.cv[c]) {
    fmin = std::min(fmin, Fs[v]);
    fmax = std::max(fmax, Fs[v]);
  }
  const real half = real(0.5);
  if (!(fmin < half && half < fmax)) return false;
  struct Seg {
    int from_a, from_b, to_a, to_b;  // edges (lower, higher vertex) of the start and end crossings
    int face;
    bool used;
  };
  std::vector<Seg> seg;
  for (auto& fs : M.cf[c]) {
    int f = fs.first, b = M.fptr[f], k = M.fptr[f + 1] - b;
    std::vector<int> vs(k);
    for (int i = 0; i < k; ++i) vs[i] = M.fidx[b + i];
    if (fs.second < 0) std::reverse(vs.begin(), vs.end());  // outward orientation of c
    int enter_a = -1, enter_b = -1, leave_a = -1, leave_b = -1, ncross = 0;
    for (int i = 0; i < k; ++i) {
      int a = vs[i], e = vs[(i + 1) % k];
      bool ia = Fs[a] >= half, ie = Fs[e] >= half;
      if (ia == ie) continue;
      ++ncross;
      if (ie) {
        enter_a = std::min(a, e);
        enter_b = std::max(a, e);
      } else {
        leave_a = std::min(a, e);
        leave_b = std::max(a, e);
      }
    }
    if (ncross == 0) continue;
    if (ncross != 2) return false;
    seg.push_back({enter_a, enter_b, leave_a, leave_b, f, false});
  }
  if (seg.size() < 3) return false;
  auto point = [&](int a, int e) {
    real t = (half - Fs[a]) / (Fs[e] - Fs[a]);
    return M.X[a] + t * (M.X[e] - M.X[a]);
  };
  size_t cur = 0;
  seg[0].used = true;
  for (size_t n = 0; n < seg.size(); ++n) {
    cyc.push_back(point(seg[cur].from_a, seg[cur].from_b));
    cface.push_back(seg[cur].face);
    if (n + 1 == seg.size()) break;
    size_t nxt = seg.size();
    for (size_t j = 0; j < seg.size(); ++j)
      if (!seg[j].used && seg[j].from_a == seg[cur].to_a && seg[j].from_b == seg[cur].to_b) {
        nxt = j;
        break;
      }
    if (nxt == seg.size()) return false;  // the loop closed early: more than one isosurface
    seg[nxt].used = true;
    cur = nxt;
  }
  // the last segment must end where the first starts
  return seg[cur].to_a == seg[0].from_a && seg[cur].to_b == seg[0].from_b;
}

V3 vmean(const std::vector<V3>& p) {
  V3 g = mk(0.0, 0.0, 0.0);
  for (auto& q : p) g = g + q;
  real k = real(double(p.size()));
  return mk(g.x / k, g.y / k, g.z / k);
}

// Area-weighted mean of the unit normals of the fan triangles (o, r_j,
// r_{j+1}) over a closed ring: the sum of the triangles' cross products.
V3 fan_normal(V3 o, const std::vector<V3>& ring) {
  V3 s = mk(0.0, 0.0, 0.0);
  size_t k = ring.size();
  for (size_t j = 0; j < k; ++j) s = s + cross(ring[j] - o, ring[(j + 1) % k] - o);
  return s;
}

// Unit vector of s, zero when s is.  The loop runs with the inside (F* >=
// 1/2) on its left as seen from the side s points to, which puts s on the
// outside; the unit normal is turned to the fluid.
V3 iso_unit(V3 s) {
  real ss = dot(s, s);
  if (ss == real(0.0)) return mk(0.0, 0.0, 0.0);
  real inv = real(-1.0) / sqrt(ss);  // turned from the outside to the fluid
  return mk(s.x * inv, s.y * inv, s.z * inv);
}

// Isosurface normals of the interfacial cells.  LLCIR: the local polygon's
// fan about its vertex mean g_c.  ELCIR: the fan about g_c over the ring
// through the polygon's points and, after the point starting each polygon
// edge, the isosurface centre g_k of the cell across the face that edge lies
// on (when that cell has an isosurface); kept only within 1.2 rad of the
// LLCIR normal.  CLCIR: after the ELCIR planes are placed, the same ring with
// g_c and the g_k replaced by the PLIC centres of those cells' planes; kept
// only within 1.2 rad of the ELCIR normal.  ok[c]: the cell has an
// isosurface (otherwise its normal stays as given, LSGIR).  level: 2 LLCIR,
// 3 ELCIR, 4 CLCIR.  On entry nrm/Cc hold the LSGIR planes.
void iso_reconstruct(const OMesh& M, const double* F, const std::vector<real>& Fs, const int8_t* tc, int level,
                     std::vector<V3>& nrm, std::vector<real>& Cc, std::vector<char>& ok) {
  const int nc = M.nc;
  const real cos12 = real(std::cos(1.2));
  std::vector<std::vector<V3>> cyc(nc);
  std::vector<std::vector<int>> cface(nc);
  std::vector<V3> g(nc, mk(0.0, 0.0, 0.0)), nl(nc, mk(0.0, 0.0, 0.0));
  ok.assign(nc, 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int c = 0; c < nc; ++c) {
    if (tc[c] != 0 || !iso_polygon(M, c, Fs, cyc[c], cface[c])) continue;
    g[c] = vmean(cyc[c]);
    V3 u = iso_unit(fan_normal(g[c], cyc[c]));
    if (dot(u, u) == real(0.0)) continue;
    nl[c] = u;
    ok[c] = 1;
  }
  auto ring_normal = [&](int c, const std::vector<V3>& cen) {
    std::vector<V3> ring;
    for (size_t i = 0; i < cyc[c].size(); ++i) {
      int f = cface[c][i];
      int k = M.owner[f] == c ? M.neigh[f] : M.owner[f];
      ring.push_back((k >= 0 && ok[k]) ? cen[k] : cyc[c][i]);
    }
    return iso_unit(fan_normal(cen[c], ring));
  };
  auto place = [&](const std::vector<V3>& nn) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < nc; ++c) {
      if (!ok[c]) continue;
      nrm[c] = nn[c];
      Cc[c] = plane_constant(M, c, nrm[c], F[c]);
    }
  };
  if (level == 2) {
    place(nl);
    return;
  }
  std::vector<V3> ne(nc, mk(0.0, 0.0, 0.0));
#pragma omp parallel for schedule(dynamic, 16)
  for (int c = 0; c < nc; ++c) {
    if (!ok[c]) continue;
    V3 u = ring_normal(c, g);
    ne[c] = (dot(u, u) > real(0.0) && dot(u, nl[c]) > cos12) ? u : nl[c];
  }
  place(ne);
  if (level == 3) return;
  std::vector<V3> x(nc, mk(0.0, 0.0, 0.0)), nk(nc, mk(0.0, 0.0, 0.0));
#pragma omp parallel for schedule(dynamic, 16)
  for (int c = 0; c < nc; ++c)
    if (ok[c]) plic_centre(M, c, nrm[c], Cc[c], x[c]);
#pragma omp parallel for schedule(dynamic, 16)
  for (int c = 0; c < nc; ++c) {
    if (!ok[c]) continue;
    V3 u = ring_normal(c, x);
    nk[c] = (dot(u, u) > real(0.0) && dot(u, ne[c]) > cos12) ? u : ne[c];
  }
  place(nk);
}

// The outer iteration (Sec. "Swartz interface reconstruction", applied to
// LSFIR): from the LSGIR planes, repeatedly take every interfacial cell's
// PLIC centre, fit each cell's normal, and adopt the fitted normal where it
// turns by less than 30/I_out degrees (I_out = 1, 2, ...), all cells at once;
// then place each changed plane to match F.  Stops after lsfir_outer passes,
// or after a pass in which no normal turned by lsfir_tol or more.
void lsfir_iterate(const OMesh& M, const double* F, const int8_t* tc, std::vector<V3>& nrm, std::vector<real>& Cc) {
  const int nc = M.nc;
  std::vector<V3> xc(nc, mk(0.0, 0.0, 0.0)), nn(nc);
  for (int it = 1; it <= M.lsfir_outer; ++it) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < nc; ++c)
      if (tc[c] == 0) plic_centre(M, c, nrm[c], Cc[c], xc[c]);
    const real lim = real(std::cos((3.14159265358979323846 / 6.0) / double(it)));  // constants
    const real stop = real(std::cos(M.lsfir_tol));
    int turned = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : turned)
    for (int c = 0; c < nc; ++c) {
      nn[c] = nrm[c];
      if (tc[c] != 0) continue;
      int nv;
      V3 e = lsfir_fit(M, c, nrm, xc, tc, nv);
      real d = dot(e, nrm[c]);
      if (d > lim) nn[c] = e;
      if (dot(nn[c], nrm[c]) < stop) ++turned;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < nc; ++c) {
      if (tc[c] != 0) continue;
      bool same = nn[c].x == nrm[c].x && nn[c].y == nrm[c].y && nn[c].z == nrm[c].z;
      nrm[c] = nn[c];
      if (!same) Cc[c] = plane_constant(M, c, nrm[c], F[c]);
    }
    if (turned == 0) break;
  }
}

// --------------------------------------------------------------------------
// FMFPA flux polyhedron (Sec. "Face-matched flux polyhedron").
//   first face = the cell face x_0..x_{I-1};
//   lateral face i contains edge (x_i, x_{i+1}) and is parallel to the
//   edge-centre velocity (u_i + u_{i+1})/2: normal m_i = (x_{i+1}-x_i) x ubar_i;
//   back vertex b_i on the line where lateral planes i-1 and i meet
//   (direction d_i = m_{i-1} x m_i), at the projection of x_i - dt u_i on
//   that line; if the two planes are (nearly) parallel, b_i = x_i - dt u_i;
//   back face triangulated about the mean g of the b_i moved along the face
//   normal (along S) so that the signed volume equals V_d.
// Tets fanned from the face centre: for each edge i,
//   (c; x_{i+1}, x_i, b_{i+1}), (c; x_i, b_i, b_{i+1}), (c; a, b_{i+1}, b_i).
// --------------------------------------------------------------------------
struct FluxPoly {
  int I = 0;
  std::vector<V3> x, b, m;  // m: EMFPA lateral-face centres (empty for FMFPA)
  V3 a, c;
  bool degenerate = false;
  std::vector<std::array<V3, 4>> tets;
  std::vector<real> sgn;
};

void fmfpa(const OMesh& M, int f, const double* uv, double dt_, real Vd, double degen, FluxPoly& P) {
  int b0 = M.fptr[f], I = M.fptr[f + 1] - b0;
  int nv = M.nv;
  real dt = dt_;
  P.I = I;
  P.x.resize(I);
  P.b.resize(I);
  std::vector<V3> u(I), m(I);
  for (int i = 0; i < I; ++i) {
    int v = M.fidx[b0 + i];
    P.x[i] = M.X[v];
    u[i] = mk(uv[v], uv[nv + v], uv[2 * nv + v]);
  }
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    V3 ub = mk(real(0.5) * (u[i].x + u[j].x), real(0.5) * (u[i].y + u[j].y), real(0.5) * (u[i].z + u[j].z));
    m[i] = cross(P.x[j] - P.x[i], ub);
  }
  for (int i = 0; i < I; ++i) {
    V3 m0 = m[(i + I - 1) % I], m1 = m[i];
    V3 d = cross(m0, m1);
    real dd = dot(d, d), a0 = dot(m0, m0), a1 = dot(m1, m1);
    bool fallback = (a0 == real(0.0)) || (a1 == real(0.0)) || (dd <= (real(degen) * a0) * a1);
    if (fallback) {
      P.b[i] = P.x[i] - dt * u[i];
    } else {
      real t = dot(u[i], d) / dd;
      P.b[i] = P.x[i] - (dt * t) * d;
    }
  }
  P.c = M.fc[f];
  V3 g = mk(0.0, 0.0, 0.0);
  for (int i = 0; i < I; ++i) g = g + P.b[i];
  real iI = real(double(I));
  g = mk(g.x / iI, g.y / iI, g.z / iI);
  V3 S = M.S[f], c = P.c;
  // signed volume with the apex at g, and its slope along S
  real V0 = 0.0, W = 0.0;
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    V0 = V0 + det3(P.x[j] - c, P.x[i] - c, P.b[j] - c);
    V0 = V0 + det3(P.x[i] - c, P.b[i] - c, P.b[j] - c);
    V0 = V0 + det3(g - c, P.b[j] - c, P.b[i] - c);
    W = W + det3(S, P.b[j] - c, P.b[i] - c);
  }
  V0 = V0 / real(6.0);
  W = W / real(6.0);
  real SS = dot(S, S);
  real mu = 0.0;
  if (fabs(W) <= real(1e-12) * SS) {
    P.degenerate = true;
  } else {
    mu = (Vd - V0) / W;
  }
  P.a = g + mu * S;
  P.tets.clear();
  P.sgn.clear();
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    std::array<V3, 4> t1 = {c, P.x[j], P.x[i], P.b[j]};
    std::array<V3, 4> t2 = {c, P.x[i], P.b[i], P.b[j]};
    std::array<V3, 4> t3 = {c, P.a, P.b[j], P.b[i]};
    for (auto* t : {&t1, &t2, &t3}) {
      real d = det3((*t)[1] - c, (*t)[2] - c, (*t)[3] - c);
      if (d == real(0.0)) continue;
      P.tets.push_back(*t);
      P.sgn.push_back(d > real(0.0) ? real(1.0) : real(-1.0));
    }
  }
}

// --------------------------------------------------------------------------
// EMFPA flux polyhedron (Sec. "Edge-matched flux polyhedron").
//   first face = the cell face x_0..x_{I-1};
//   back vertex b_i = x_i - dt u_i: vertex i moved back along its streak line,
//   Eq. (streak-line2), so every face through a vertex shares its b_i;
//   lateral face i, bounded by x_i, x_{i+1}, b_{i+1}, b_i, is replaced by four
//   triangles about its vertex mean m_i (3I+1 vertices in all);
//   back face triangulated about the mean g of the b_i moved along the face
//   normal (along S) so that the signed volume equals V_d (5I+1 faces).
// m_i sums the two edge ends and the two back vertices pairwise, an order
// symmetric in i and i+1, so the faces on either side of an edge build the
// same centre to the last bit.
// Tets fanned from the face centre: for each edge i (j = i+1),
//   (c; x_j, x_i, m_i), (c; x_i, b_i, m_i), (c; b_i, b_j, m_i), (c; b_j, x_j, m_i),
//   (c; a, b_j, b_i)
// (the lateral quad taken x_j, x_i, b_i, b_j: the orientation of the FMFPA
// lateral face).
// --------------------------------------------------------------------------
void emfpa(const OMesh& M, int f, const double* uv, double dt_, real Vd, FluxPoly& P) {
  int b0 = M.fptr[f], I = M.fptr[f + 1] - b0;
  int nv = M.nv;
  real dt = dt_;
  P.I = I;
  P.x.resize(I);
  P.b.resize(I);
  P.m.resize(I);
  for (int i = 0; i < I; ++i) {
    int v = M.fidx[b0 + i];
    P.x[i] = M.X[v];
    V3 u = mk(uv[v], uv[nv + v], uv[2 * nv + v]);
    P.b[i] = P.x[i] - dt * u;
  }
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    V3 s = (P.x[i] + P.x[j]) + (P.b[i] + P.b[j]);
    P.m[i] = mk(s.x / real(4.0), s.y / real(4.0), s.z / real(4.0));
  }
  P.c = M.fc[f];
  V3 g = mk(0.0, 0.0, 0.0);
  for (int i = 0; i < I; ++i) g = g + P.b[i];
  real iI = real(double(I));
  g = mk(g.x / iI, g.y / iI, g.z / iI);
  V3 S = M.S[f], c = P.c;
  // signed volume with the back-face vertex at g, and its slope along S
  real V0 = 0.0, W = 0.0;
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    V3 xi = P.x[i] - c, xj = P.x[j] - c, bi = P.b[i] - c, bj = P.b[j] - c, mi = P.m[i] - c;
    V0 = V0 + det3(xj, xi, mi);
    V0 = V0 + det3(xi, bi, mi);
    V0 = V0 + det3(bi, bj, mi);
    V0 = V0 + det3(bj, xj, mi);
    V0 = V0 + det3(g - c, bj, bi);
    W = W + det3(S, bj, bi);
  }
  V0 = V0 / real(6.0);
  W = W / real(6.0);
  real SS = dot(S, S);
  real mu = 0.0;
  if (fabs(W) <= real(1e-12) * SS) {
    P.degenerate = true;
  } else {
    mu = (Vd - V0) / W;
  }
  P.a = g + mu * S;
  P.tets.clear();
  P.sgn.clear();
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    std::array<V3, 4> t[5] = {{c, P.x[j], P.x[i], P.m[i]},
                              {c, P.x[i], P.b[i], P.m[i]},
                              {c, P.b[i], P.b[j], P.m[i]},
                              {c, P.b[j], P.x[j], P.m[i]},
                              {c, P.a, P.b[j], P.b[i]}};
    for (auto& T : t) {
      real d = det3(T[1] - c, T[2] - c, T[3] - c);
      if (d == real(0.0)) continue;
      P.tets.push_back(T);
      P.sgn.push_back(d > real(0.0) ? real(1.0) : real(-1.0));
    }
  }
}

// --------------------------------------------------------------------------
// NMFPA flux polyhedron (Sec. "Non-matched flux polyhedron").
//   every vertex of the face moves back with the one face-centre velocity
//   u_f: b_i = x_i - dt u_f (Eq. streak-line2 with u_f for every vertex);
//   each lateral face (x_i, x_{i+1}, b_{i+1}, b_i) is then a planar
//   parallelogram and the back face the translated cell face, so the
//   polyhedron (I+2 faces, 2I vertices) has volume dt u_f.S = V_d with no
//   adjustment.
// Tets fanned from the face centre: for each edge i (j = i+1),
//   (c; x_j, x_i, b_j), (c; x_i, b_i, b_j) (the FMFPA lateral split), and the
//   planar back face fanned from b_0: (c; b_0, b_{k+1}, b_k), k = 1..I-2.
// --------------------------------------------------------------------------
void nmfpa(const OMesh& M, int f, const double* uf, double dt_, FluxPoly& P) {
  int b0 = M.fptr[f], I = M.fptr[f + 1] - b0;
  int nf = M.nf;
  real dt = dt_;
  V3 u = mk(uf[f], uf[nf + f], uf[2 * nf + f]);
  P.I = I;
  P.x.resize(I);
  P.b.resize(I);
  for (int i = 0; i < I; ++i) {
    P.x[i] = M.X[M.fidx[b0 + i]];
    P.b[i] = P.x[i] - dt * u;
  }
  P.c = M.fc[f];
  P.a = P.b[0];
  V3 c = P.c;
  P.tets.clear();
  P.sgn.clear();
  std::vector<std::array<V3, 4>> t;
  for (int i = 0; i < I; ++i) {
    int j = (i + 1) % I;
    t.push_back({c, P.x[j], P.x[i], P.b[j]});
    t.push_back({c, P.x[i], P.b[i], P.b[j]});
  }
  for (int k = 1; k + 1 < I; ++k) t.push_back({c, P.b[0], P.b[k + 1], P.b[k]});
  for (auto& T : t) {
    real d = det3(T[1] - c, T[2] - c, T[3] - c);
    if (d == real(0.0)) continue;
    P.tets.push_back(T);
    P.sgn.push_back(d > real(0.0) ? real(1.0) : real(-1.0));
  }
}

// The flux polyhedron of face f by the mesh's method (uf: face velocities,
// read by NMFPA only).
void flux_poly(const OMesh& M, int f, const double* uf, const double* uv, double dt, real Vd, double degen,
               FluxPoly& P) {
  if (M.method == 1) emfpa(M, f, uv, dt, Vd, P);
  else if (M.method == 2) nmfpa(M, f, uf, dt, P);
  else fmfpa(M, f, uv, dt, Vd, degen, P);
}

// Candidate cells of face f: the owner, the neighbour and every cell sharing
// a vertex with either of them, ascending.
void candidates(const OMesh& M, int f, std::vector<int>& out) {
  out.clear();
  int o = M.owner[f], n = M.neigh[f];
  out.push_back(o);
  for (int k : M.nb[o]) out.push_back(k);
  if (n >= 0) {
    out.push_back(n);
    for (int k : M.nb[n]) out.push_back(k);
  }
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
}

// Whether the flux polyhedron of face f stays within the cells the
// truncation visits (the candidates; "donating regions from several cells",
// Sec. "Fluid advected through cell faces"): every point it is built from
// (x_i, b_i, the apex, the face centre, EMFPA's lateral centres) lies in the
// closed enclosing box of some candidate cell, or outside the enclosing box
// of the whole mesh (outside the domain, which holds no fluid).  The
// polyhedron lies in the convex hull of these points, so on a Cartesian grid,
// whose candidates' boxes tile one box, this is exact; elsewhere it tests
// boxes, not cells.
bool flux_covered(const OMesh& M, int f, const FluxPoly& P) {
  std::vector<int> cand;
  candidates(M, f, cand);
  std::vector<V3> pts(P.x);
  pts.insert(pts.end(), P.b.begin(), P.b.end());
  pts.insert(pts.end(), P.m.begin(), P.m.end());
  pts.push_back(P.a);
  pts.push_back(P.c);
  auto in_box = [](V3 p, V3 lo, V3 hi) {
    return lo.x <= p.x && p.x <= hi.x && lo.y <= p.y && p.y <= hi.y && lo.z <= p.z && p.z <= hi.z;
  };
  for (V3 p : pts) {
    if (!in_box(p, M.dom_lo, M.dom_hi)) continue;
    bool in = false;
    for (int k : cand) in = in || in_box(p, M.bbmin[k], M.bbmax[k]);
    if (!in) return false;
  }
  return true;
}

// V_F of a tag-0 face: signed truncation of the flux polyhedron by the fluid
// of every candidate cell (full cells whole, interfacial cells by their PLIC
// half-space, empty cells skipped).
real face_fluid_volume(const OMesh& M, int f, const FluxPoly& P, const double* planes, const int8_t* tcell) {
  std::vector<int> cand;
  candidates(M, f, cand);
  int nc = M.nc;
  real acc = 0.0;
  for (size_t t = 0; t < P.tets.size(); ++t) {
    const V3* T = P.tets[t].data();
    real part = 0.0;
    for (int k : cand) {
      if (tcell[k] == -1) continue;
      bool plane = tcell[k] == 0;
      V3 n = mk(planes[k], planes[nc + k], planes[2 * nc + k]);
      real C = planes[3 * nc + k];
      part = part + tet_cell_volume(M, T, k, plane, n, C);
    }
    acc = acc + P.sgn[t] * part;
  }
  return acc;
}

struct FaceOut {
  real Vd, VF;
  int up;
  bool degenerate;
};

FaceOut face_flux(const OMesh& M, int f, const double* planes, const int8_t* tcell, const int8_t* tface,
                  const double* uf, const double* uv, double dt, double degen) {
  FaceOut o{0.0, 0.0, -1, false};
  int nf = M.nf;
  V3 S = M.S[f];
  V3 u = mk(uf[f], uf[nf + f], uf[2 * nf + f]);
  o.Vd = real(dt) * dot(u, S);
  o.up = o.Vd >= real(0.0) ? M.owner[f] : M.neigh[f];
  if (M.neigh[f] < 0 && o.Vd < real(0.0)) o.VF = 0.0;  // inflow from an empty outside
  else if (tface[f] == -1) o.VF = 0.0;
  else if (tface[f] == 1) o.VF = o.Vd;
  else {
    FluxPoly P;
    flux_poly(M, f, uf, uv, dt, o.Vd, degen, P);
    o.degenerate = P.degenerate;
    o.VF = face_fluid_volume(M, f, P, planes, tcell);
  }
  return o;
}

// Eq. (fnext) followed by the clamp to [0, 1].
real update_cell(const OMesh& M, int c, const double* Vd, const double* VF, double Fin) {
  real VdT = 0.0, VFT = 0.0;
  for (auto& fs : M.cf[c]) {
    real sg = real(double(fs.second));
    VdT = VdT + sg * real(Vd[fs.first]);
    VFT = VFT + sg * real(VF[fs.first]);
  }
  real V = M.V[c];
  real h = VdT / (real(2.0) * V);
  real Fn = (real(Fin) * (real(1.0) + h) - VFT / V) / (real(1.0) - h);
  if (Fn > real(1.0)) Fn = 1.0;
  if (Fn < real(0.0)) Fn = 0.0;
  return Fn;
}

// --------------------------------------------------------------------------
// Refinement initialisation: an n_div^3 grid of sub-boxes over the cell's
// enclosing box.  Sub-box with all eight corners inside the body -> its part
// inside the cell counts whole; all outside -> nothing; otherwise its part
// inside the cell is cut by the body's tangent plane at the sub-box centre.
// shape 0: sphere (cx, cy, cz, r), inside |x - c| <= r.
// shape 1: half-space (nx, ny, nz, C), inside n.x + C >= 0.
// --------------------------------------------------------------------------
inline bool inside(int shape, const double* sp, V3 p) {
  if (shape == 0) {
    V3 d = p - mk(sp[0], sp[1], sp[2]);
    return (d.x * d.x + d.y * d.y) + d.z * d.z <= real(sp[3]) * real(sp[3]);
  }
  return dot(mk(sp[0], sp[1], sp[2]), p) + real(sp[3]) >= real(0.0);
}

real cell_box_plane_volume(const OMesh& M, int c, V3 lo, V3 hi, bool use_plane, V3 n, real C) {
  if (M.isbox[c]) {
    Poly P = box_poly(lo, hi);
    if (use_plane) clip(P, n, C);
    return volume(P);
  }
  real acc = 0.0;
  for (const Tet& t : M.tets[c]) {
    V3 tlo, thi;
    tet_bbox(t.p, tlo, thi);
    if (!boxes_overlap(tlo, thi, lo, hi)) continue;
    Plane pl[4];
    tet_planes(t.p[0], t.p[1], t.p[2], t.p[3], pl);
    Poly P = box_poly(lo, hi);
    for (int i = 0; i < 4; ++i) clip(P, pl[i].n, pl[i].d);
    if (use_plane) clip(P, n, C);
    acc = acc + t.sign * volume(P);
  }
  return acc;
}

real init_cell(const OMesh& M, int c, int shape, const double* sp, int ndiv) {
  bool allin = true, allout = true;
  for (int v : M.cv[c]) {
    if (inside(shape, sp, M.X[v])) allout = false;
    else allin = false;
  }
  if (allin) return 1.0;
  V3 lo = M.bbmin[c], hi = M.bbmax[c];
  if (allout) {
    if (shape == 1) return 0.0;
    V3 ctr = mk(sp[0], sp[1], sp[2]);
    V3 q = mk(std::min(std::max(ctr.x, lo.x), hi.x), std::min(std::max(ctr.y, lo.y), hi.y),
              std::min(std::max(ctr.z, lo.z), hi.z));
    V3 d = ctr - q;
    if ((d.x * d.x + d.y * d.y) + d.z * d.z > real(sp[3]) * real(sp[3])) return 0.0;
  }
  real nd = real(double(ndiv));
  V3 hs = mk((hi.x - lo.x) / nd, (hi.y - lo.y) / nd, (hi.z - lo.z) / nd);
  real acc = 0.0;
  for (int kz = 0; kz < ndiv; ++kz)
    for (int ky = 0; ky < ndiv; ++ky)
      for (int kx = 0; kx < ndiv; ++kx) {
        V3 a = mk(lo.x + real(double(kx)) * hs.x, lo.y + real(double(ky)) * hs.y, lo.z + real(double(kz)) * hs.z);
        V3 b = mk(lo.x + real(double(kx + 1)) * hs.x, lo.y + real(double(ky + 1)) * hs.y,
                  lo.z + real(double(kz + 1)) * hs.z);
        int nin = 0;
        for (int q = 0; q < 8; ++q) {
          V3 p = mk((q & 1) ? b.x : a.x, (q & 2) ? b.y : a.y, (q & 4) ? b.z : a.z);
          if (inside(shape, sp, p)) ++nin;
        }
        if (nin == 0) continue;
        if (nin == 8) {
          acc = acc + cell_box_plane_volume(M, c, a, b, false, mk(0.0, 0.0, 0.0), 0.0);
          continue;
        }
        V3 n;
        real C;
        if (shape == 0) {
          V3 cs = mk(real(0.5) * (a.x + b.x), real(0.5) * (a.y + b.y), real(0.5) * (a.z + b.z));
          V3 r = cs - mk(sp[0], sp[1], sp[2]);
          real rl = sqrt(dot(r, r));
          if (rl == real(0.0)) {
            acc = acc + cell_box_plane_volume(M, c, a, b, false, mk(0.0, 0.0, 0.0), 0.0);
            continue;
          }
          // phi(x) ~ (R - |cs - x0|) - (r/|r|).(x - cs) >= 0
          n = mk(-r.x / rl, -r.y / rl, -r.z / rl);
          C = (real(sp[3]) - rl) - dot(n, cs);
        } else {
          n = mk(sp[0], sp[1], sp[2]);
          C = sp[3];
        }
        acc = acc + cell_box_plane_volume(M, c, a, b, true, n, C);
      }
  return acc / M.V[c];
}

}  // namespace

// ==========================================================================
// C interface (ctypes).  Arrays of 3- or 4-vectors are structure-of-arrays:
// component k of item i at [k * count + i].
// ==========================================================================
extern "C" {

int orc_counting_build() {
#ifdef ORC_COUNT_FLOPS
  return 1;
#else
  return 0;
#endif
}
long long orc_flops_get() {
#ifdef ORC_COUNT_FLOPS
  return g_orc_flops;
#else
  return -1;
#endif
}
void orc_flops_reset() {
#ifdef ORC_COUNT_FLOPS
  g_orc_flops = 0;
#endif
}

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void* orc_mesh_new(int nv, const double* vx, const double* vy, const double* vz, int nf, const int* fptr,
                   const int* fidx, const int* owner, const int* neigh, int nc) {
  OMesh* M = new OMesh;
  M->nv = nv;
  M->nf = nf;
  M->nc = nc;
  M->X.resize(nv);
  for (int i = 0; i < nv; ++i) M->X[i] = mk(vx[i], vy[i], vz[i]);
  M->fptr.assign(fptr, fptr + nf + 1);
  M->fidx.assign(fidx, fidx + fptr[nf]);
  M->owner.assign(owner, owner + nf);
  M->neigh.assign(neigh, neigh + nf);
  build_mesh(*M);
  return M;
}

void orc_mesh_free(void* h) { delete static_cast<OMesh*>(h); }

// Normals of the mesh's reconstruction: 0 LSGIR (default), 1 LSFIR with at
// most `outer` outer iterations and stopping tolerance tol (rad), the weight
// floored at 0.05 h when cap is nonzero, 2 LLCIR, 3 ELCIR, 4 CLCIR.  Returns
// 0, or -1 for a bad value.
int orc_mesh_set_recon(void* h, int method, int outer, double tol, int cap) {
  if (method < 0 || method > 4 || outer < 1 || !(tol >= 0.0)) return -1;
  OMesh& M = *static_cast<OMesh*>(h);
  M.recon = method;
  M.lsfir_outer = outer;
  M.lsfir_tol = tol;
  M.lsfir_cap = cap != 0;
  return 0;
}

// Isosurface of F* = 1/2 in cell c from the given node values (nv): the
// polygon's points in loop order (3 doubles each, at most cap points) and the
// face of each polygon edge.  Returns the number of points, or -1 when the
// cell has no usable isosurface.
int orc_iso_polygon(void* h, int c, const double* Fs_in, int cap, double* pts, int* faces) {
  OMesh& M = *static_cast<OMesh*>(h);
  std::vector<real> Fs(M.nv);
  for (int v = 0; v < M.nv; ++v) Fs[v] = Fs_in[v];
  std::vector<V3> cyc;
  std::vector<int> cf;
  if (!iso_polygon(M, c, Fs, cyc, cf)) return -1;
  int n = (int)cyc.size();
  for (int i = 0; i < n && i < cap; ++i) {
    pts[3 * i] = to_double(cyc[i].x); pts[3 * i + 1] = to_double(cyc[i].y); pts[3 * i + 2] = to_double(cyc[i].z);
    faces[i] = cf[i];
  }
  return n;
}

// Isosurface-based planes (level 2 LLCIR, 3 ELCIR, 4 CLCIR) from given node
// values (nv), cell values F (nc, after the cut-off), tags and LSGIR planes
// (4 x nc, replaced in place for the cells with an isosurface; ok (nc) = 1
// for those).
void orc_iso_planes(void* h, const double* Fs_in, const double* F, const int8_t* tc, int level, double* planes,
                    int8_t* ok_out) {
  OMesh& M = *static_cast<OMesh*>(h);
  int nc = M.nc;
  std::vector<real> Fs(M.nv);
  for (int v = 0; v < M.nv; ++v) Fs[v] = Fs_in[v];
  std::vector<V3> nrm(nc);
  std::vector<real> Cc(nc);
  for (int c = 0; c < nc; ++c) {
    nrm[c] = mk(planes[c], planes[nc + c], planes[2 * nc + c]);
    Cc[c] = planes[3 * nc + c];
  }
  std::vector<char> ok;
  iso_reconstruct(M, F, Fs, tc, level, nrm, Cc, ok);
  for (int c = 0; c < nc; ++c) {
    planes[c] = to_double(nrm[c].x); planes[nc + c] = to_double(nrm[c].y); planes[2 * nc + c] = to_double(nrm[c].z);
    planes[3 * nc + c] = to_double(Cc[c]);
    ok_out[c] = ok[c];
  }
}

// PLIC centres (3 x nc) of the tag-0 cells for the given planes (4 x nc);
// other cells get 0.  cnt (nc) receives the number of polygon vertices.
void orc_plic_centres(void* h, const int8_t* tc, const double* planes, double* out, int* cnt) {
  OMesh& M = *static_cast<OMesh*>(h);
  int nc = M.nc;
  for (int c = 0; c < nc; ++c) {
    out[c] = out[nc + c] = out[2 * nc + c] = 0.0;
    cnt[c] = 0;
    if (tc[c] != 0) continue;
    V3 x;
    cnt[c] = plic_centre(M, c, mk(planes[c], planes[nc + c], planes[2 * nc + c]), planes[3 * nc + c], x);
    out[c] = to_double(x.x); out[nc + c] = to_double(x.y); out[2 * nc + c] = to_double(x.z);
  }
}

// One LSFIR fit of every tag-0 cell from the given normals (3 x nc) and PLIC
// centres (3 x nc): fitted normals (3 x nc, before the outer iteration's
// turn limit) and the number of valid neighbours (nc).
void orc_lsfir_fit(void* h, const int8_t* tc, const double* normals, const double* centres, double* out,
                   int* nvalid) {
  OMesh& M = *static_cast<OMesh*>(h);
  int nc = M.nc;
  std::vector<V3> nrm(nc), xc(nc);
  for (int c = 0; c < nc; ++c) {
    nrm[c] = mk(normals[c], normals[nc + c], normals[2 * nc + c]);
    xc[c] = mk(centres[c], centres[nc + c], centres[2 * nc + c]);
  }
  for (int c = 0; c < nc; ++c) {
    out[c] = out[nc + c] = out[2 * nc + c] = 0.0;
    nvalid[c] = 0;
    if (tc[c] != 0) continue;
    V3 e = lsfir_fit(M, c, nrm, xc, tc, nvalid[c]);
    out[c] = to_double(e.x); out[nc + c] = to_double(e.y); out[2 * nc + c] = to_double(e.z);
  }
}

// Flux polyhedra of the mesh: 0 FMFPA (default), 1 EMFPA, 2 NMFPA.  Returns
// 0, or -1 for another value.
int orc_mesh_set_method(void* h, int method) {
  if (method < 0 || method > 2) return -1;
  static_cast<OMesh*>(h)->method = method;
  return 0;
}

void orc_geometry(void* h, double* S, double* fc, double* V, double* cc, double* bbmin, double* bbmax,
                  int8_t* isbox) {
  OMesh& M = *static_cast<OMesh*>(h);
  for (int f = 0; f < M.nf; ++f) {
    S[f] = to_double(M.S[f].x); S[M.nf + f] = to_double(M.S[f].y); S[2 * M.nf + f] = to_double(M.S[f].z);
    fc[f] = to_double(M.fc[f].x); fc[M.nf + f] = to_double(M.fc[f].y); fc[2 * M.nf + f] = to_double(M.fc[f].z);
  }
  for (int c = 0; c < M.nc; ++c) {
    V[c] = to_double(M.V[c]);
    cc[c] = to_double(M.cc[c].x); cc[M.nc + c] = to_double(M.cc[c].y); cc[2 * M.nc + c] = to_double(M.cc[c].z);
    bbmin[c] = to_double(M.bbmin[c].x); bbmin[M.nc + c] = to_double(M.bbmin[c].y);
    bbmin[2 * M.nc + c] = to_double(M.bbmin[c].z);
    bbmax[c] = to_double(M.bbmax[c].x); bbmax[M.nc + c] = to_double(M.bbmax[c].y);
    bbmax[2 * M.nc + c] = to_double(M.bbmax[c].z);
    isbox[c] = M.isbox[c];
  }
}

// Vertex-sharing neighbour lists as CSR; returns the total count (call with
// idx = nullptr to size).
int orc_neighbours(void* h, int* ptr, int* idx) {
  OMesh& M = *static_cast<OMesh*>(h);
  int n = 0;
  for (int c = 0; c < M.nc; ++c) {
    if (ptr) ptr[c] = n;
    for (int k : M.nb[c]) {
      if (idx) idx[n] = k;
      ++n;
    }
  }
  if (ptr) ptr[M.nc] = n;
  return n;
}

void orc_tags(void* h, const double* F, double eps, double* Fstar, int8_t* tn, int8_t* tf, int8_t* tc) {
  OMesh& M = *static_cast<OMesh*>(h);
  std::vector<real> Fs;
  tags(M, F, eps, Fs, tn, tf, tc);
  for (int v = 0; v < M.nv; ++v) Fstar[v] = to_double(Fs[v]);
}

// Normals of the tag-0 cells from (already cut-off) F.
void orc_lsgir(void* h, const double* F, const int8_t* tc, double beta, double* n) {
  OMesh& M = *static_cast<OMesh*>(h);
#pragma omp parallel for schedule(dynamic, 64)
  for (int c = 0; c < M.nc; ++c) {
    V3 v = mk(0.0, 0.0, 0.0);
    if (tc[c] == 0) v = lsgir_normal(M, F, c, beta);
    n[c] = to_double(v.x); n[M.nc + c] = to_double(v.y); n[2 * M.nc + c] = to_double(v.z);
  }
}

void orc_plane_constant(void* h, const double* F, const int8_t* tc, const double* n, double* C) {
  OMesh& M = *static_cast<OMesh*>(h);
#pragma omp parallel for schedule(dynamic, 16)
  for (int c = 0; c < M.nc; ++c) {
    C[c] = 0.0;
    if (tc[c] != 0) continue;
    C[c] = to_double(plane_constant(M, c, mk(n[c], n[M.nc + c], n[2 * M.nc + c]), F[c]));
  }
}

double orc_cell_cut_volume(void* h, int c, double nx, double ny, double nz, double C) {
  OMesh& M = *static_cast<OMesh*>(h);
  return to_double(cell_level_volume(M, c, mk(nx, ny, nz), -real(C)));
}

// Reconstruction: tags from the incoming F, cut-off in place, LSGIR normal
// and plane constant of every tag-0 cell.  planes: 4 x nc (nx, ny, nz, C),
// zero for cells that are not tag 0.
void orc_reconstruct(void* h, double* F, double eps, double beta, double* Fstar, int8_t* tn, int8_t* tf,
                     int8_t* tc, double* planes) {
  OMesh& M = *static_cast<OMesh*>(h);
  int nc = M.nc;
  std::vector<real> Fs;
  tags(M, F, eps, Fs, tn, tf, tc);
  if (Fstar)
    for (int v = 0; v < M.nv; ++v) Fstar[v] = to_double(Fs[v]);
  for (int c = 0; c < nc; ++c) {
    if (real(F[c]) < real(eps)) F[c] = 0.0;
    else if (real(F[c]) > real(1.0) - real(eps)) F[c] = 1.0;
  }
  std::vector<V3> nrm(nc, mk(0.0, 0.0, 0.0));
  std::vector<real> Cc(nc, real(0.0));
#pragma omp parallel for schedule(dynamic, 16)
  for (int c = 0; c < nc; ++c) {
    if (tc[c] != 0) continue;
    nrm[c] = lsgir_normal(M, F, c, beta);
    Cc[c] = plane_constant(M, c, nrm[c], F[c]);
  }
  if (M.recon == 1) lsfir_iterate(M, F, tc, nrm, Cc);
  if (M.recon >= 2) {
    std::vector<char> ok;
    iso_reconstruct(M, F, Fs, tc, M.recon, nrm, Cc, ok);
  }
  for (int c = 0; c < nc; ++c) {
    planes[c] = to_double(nrm[c].x); planes[nc + c] = to_double(nrm[c].y); planes[2 * nc + c] = to_double(nrm[c].z);
    planes[3 * nc + c] = to_double(Cc[c]);
  }
}

// Flux of selected faces (all faces when nsel < 0).  Returns the number of
// faces whose apex could not be placed (volume slope ~ 0).
int orc_face_flux(void* h, const double* planes, const int8_t* tc, const int8_t* tf, const double* uf,
                  const double* uv, double dt, double degen, int nsel, const int* sel, double* Vd, double* VF,
                  int* up) {
  OMesh& M = *static_cast<OMesh*>(h);
  int n = nsel < 0 ? M.nf : nsel;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : bad)
  for (int i = 0; i < n; ++i) {
    int f = nsel < 0 ? i : sel[i];
    FaceOut o = face_flux(M, f, planes, tc, tf, uf, uv, dt, degen);
    Vd[i] = to_double(o.Vd);
    VF[i] = to_double(o.VF);
    up[i] = o.up;
    if (o.degenerate) ++bad;
  }
  return bad;
}

// Coverage of the flux polyhedra of a step (flux_covered): uncovered[f] = 1
// for each face that builds a polyhedron (tag 0, not an inflow boundary face)
// whose polyhedron leaves its candidate cells, else 0.  Returns their number.
int orc_flux_coverage(void* h, const int8_t* tf, const double* uf, const double* uv, double dt, double degen,
                      int8_t* uncovered) {
  OMesh& M = *static_cast<OMesh*>(h);
  int n = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n)
  for (int f = 0; f < M.nf; ++f) {
    uncovered[f] = 0;
    V3 u = mk(uf[f], uf[M.nf + f], uf[2 * M.nf + f]);
    real Vd = real(dt) * dot(u, M.S[f]);
    if (tf[f] != 0 || (M.neigh[f] < 0 && Vd < real(0.0))) continue;
    FluxPoly P;
    flux_poly(M, f, uf, uv, dt, Vd, degen, P);
    if (!flux_covered(M, f, P)) {
      uncovered[f] = 1;
      ++n;
    }
  }
  return n;
}

// One advection step over the whole mesh (faceflux + vofadv).
int orc_advect(void* h, const double* planes, const int8_t* tc, const int8_t* tf, const double* uf,
               const double* uv, double dt, double degen, const double* Fin, double* Fout, double* Vd, double* VF,
               int* up) {
  OMesh& M = *static_cast<OMesh*>(h);
  int bad = orc_face_flux(h, planes, tc, tf, uf, uv, dt, degen, -1, nullptr, Vd, VF, up);
#pragma omp parallel for schedule(static)
  for (int c = 0; c < M.nc; ++c) Fout[c] = to_double(update_cell(M, c, Vd, VF, Fin[c]));
  return bad;
}

void orc_update(void* h, const double* Vd, const double* VF, const double* Fin, double* Fout) {
  OMesh& M = *static_cast<OMesh*>(h);
  for (int c = 0; c < M.nc; ++c) Fout[c] = to_double(update_cell(M, c, Vd, VF, Fin[c]));
}

// The flux polyhedron of face f by the mesh's method: points x_0..x_{I-1},
// b_0..b_{I-1}, apex (NMFPA: b_0 again, the back face's fan vertex), then
// (EMFPA) the lateral-face centres m_0..m_{I-1}; returns I (or -I when the
// apex is degenerate).  pts holds 3*(2I+1) doubles (3*(3I+1) for EMFPA, xyz
// interleaved); vol_out gets the signed volume of the tet fan.  uf (face
// velocities) is read by NMFPA only, uv (vertex velocities) by the others.
int orc_flux_polyhedron(void* h, int f, const double* uf, const double* uv, double dt, double Vd, double degen,
                        double* pts, double* vol_out) {
  OMesh& M = *static_cast<OMesh*>(h);
  FluxPoly P;
  flux_poly(M, f, uf, uv, dt, Vd, degen, P);
  int I = P.I;
  for (size_t i = 0; i < P.m.size(); ++i) {
    double* q = pts + 3 * (2 * I + 1 + i);
    q[0] = to_double(P.m[i].x); q[1] = to_double(P.m[i].y); q[2] = to_double(P.m[i].z);
  }
  for (int i = 0; i < I; ++i) {
    pts[3 * i] = to_double(P.x[i].x); pts[3 * i + 1] = to_double(P.x[i].y); pts[3 * i + 2] = to_double(P.x[i].z);
    pts[3 * (I + i)] = to_double(P.b[i].x); pts[3 * (I + i) + 1] = to_double(P.b[i].y);
    pts[3 * (I + i) + 2] = to_double(P.b[i].z);
  }
  pts[6 * I] = to_double(P.a.x); pts[6 * I + 1] = to_double(P.a.y); pts[6 * I + 2] = to_double(P.a.z);
  real v = 0.0;
  for (size_t t = 0; t < P.tets.size(); ++t) {
    auto& T = P.tets[t];
    v = v + det3(T[1] - T[0], T[2] - T[0], T[3] - T[0]);
  }
  *vol_out = to_double(v / real(6.0));
  return P.degenerate ? -I : I;
}

// vol(tet ∩ planes); tet = 12 doubles (4 points xyz), planes = 4 doubles each (n, d) for n.x + d >= 0.
double orc_tet_clip_volume(const double* tet, int np, const double* pl) {
  Poly P = tet_poly(mk(tet[0], tet[1], tet[2]), mk(tet[3], tet[4], tet[5]), mk(tet[6], tet[7], tet[8]),
                    mk(tet[9], tet[10], tet[11]));
  for (int i = 0; i < np; ++i) clip(P, mk(pl[4 * i], pl[4 * i + 1], pl[4 * i + 2]), pl[4 * i + 3]);
  return to_double(volume(P));
}

double orc_box_clip_volume(const double* lo, const double* hi, int np, const double* pl) {
  Poly P = box_poly(mk(lo[0], lo[1], lo[2]), mk(hi[0], hi[1], hi[2]));
  for (int i = 0; i < np; ++i) clip(P, mk(pl[4 * i], pl[4 * i + 1], pl[4 * i + 2]), pl[4 * i + 3]);
  return to_double(volume(P));
}

// vol(tet T ∩ cell c [∩ plane]) -- for pins on non-convex cells.
double orc_tet_cell_volume(void* h, const double* tet, int c, int use_plane, double nx, double ny, double nz,
                           double C) {
  OMesh& M = *static_cast<OMesh*>(h);
  V3 T[4] = {mk(tet[0], tet[1], tet[2]), mk(tet[3], tet[4], tet[5]), mk(tet[6], tet[7], tet[8]),
             mk(tet[9], tet[10], tet[11])};
  return to_double(tet_cell_volume(M, T, c, use_plane != 0, mk(nx, ny, nz), C));
}

void orc_init_fraction(void* h, int shape, const double* sp, int ndiv, double* F) {
  OMesh& M = *static_cast<OMesh*>(h);
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < M.nc; ++c) F[c] = to_double(init_cell(M, c, shape, sp, ndiv));
}

}  // extern "C"
