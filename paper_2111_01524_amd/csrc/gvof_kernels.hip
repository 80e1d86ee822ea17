// gVOF hot path on gfx950: grid geometry, tagging + cut-off, LSGIR + plane
// constant, face flux volumes, FMFPA or EMFPA flux polyhedra with signed
// truncation,
// and the volume-fraction update (Lopez & Hernandez, arXiv 2111.01524).
//
// Sweeps over faces / cells / vertices use one lane per item in coalesced SoA
// order.  Interfacial cells and faces are compacted into work lists with
// wave-aggregated atomics; the geometric kernels walk those lists.  No
// floating-point atomics: every sum has a fixed order, so results are
// reproducible run to run.
#include <hip/hip_runtime.h>

#include <mutex>

#include "clip.h"
#include "units.h"
#include "gvof_dev.h"
#include "gvof_launch.h"

namespace gvof {

__device__ inline int grid_stride_start() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int grid_stride() { return gridDim.x * blockDim.x; }

// Wave-aggregated append of `item` when `pred`: one atomic per wave, slots in lane order.
__device__ inline void wave_append(bool pred, int item, int* counter, int* list, unsigned long long* total = nullptr) {
  unsigned long long m = __ballot(pred);
  if (m == 0) return;
  int lane = __lane_id();
  int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) {
    base = atomicAdd(counter, __popcll(m));
    if (total) atomicAdd(total, (unsigned long long)__popcll(m));
  }
  base = __shfl(base, leader);
  if (pred) {
    unsigned long long below = m & ((1ull << lane) - 1ull);
    list[base + __popcll(below)] = item;
  }
}

// Block-aggregated append of `item` when `pred`: one atomic per block (a
// counter shared by every wave of the grid is the bottleneck of a sweep
// otherwise), slots in (wave, lane) order within the block.  Every thread of
// the block must make the same number of calls: it holds block barriers.
constexpr int kMaxBlockWaves = 16;
__device__ inline void block_append(bool pred, int item, int* counter, int* list, unsigned long long* total) {
  __shared__ int s_off[kMaxBlockWaves];
  __shared__ int s_base;
  const int lane = __lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long m = __ballot(pred);
  if (lane == 0) s_off[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < nw; ++i) {
      int c = s_off[i];
      s_off[i] = t;
      t += c;
    }
    s_base = t ? atomicAdd(counter, t) : 0;
    if (total && t) atomicAdd(total, (unsigned long long)t);
  }
  __syncthreads();
  if (pred) list[s_base + s_off[w] + __popcll(m & ((1ull << lane) - 1ull))] = item;
  __syncthreads();  // s_off and s_base are reused by the next call
}

__global__ void k_zero(int* p, int n) {
  int i = grid_stride_start();
  if (i < n) p[i] = 0;
}

// ============================================================== grid geometry
// Face vertex mean c and area vector S = 1/2 sum (x_i - c) x (x_{i+1} - c),
// evaluated in vertex order with separate roundings (bitwise reproducible).
__global__ void k_face_geom(DevMesh M) {
  for (int f = grid_stride_start(); f < M.nf; f += grid_stride()) {
    int b = fv_begin(M, f), k = fv_count(M, f);
    d3 s = mk3(0.0, 0.0, 0.0);
    for (int i = 0; i < k; ++i) s = s + vert(M, M.fv_idx[b + i]);
    double dk = (double)k;
    d3 c = mk3(s.x / dk, s.y / dk, s.z / dk);
    d3 A = mk3(0.0, 0.0, 0.0);
    for (int i = 0; i < k; ++i) {
      int j = (i + 1 == k) ? 0 : i + 1;
      A = A + cross_x(vert(M, M.fv_idx[b + i]) - c, vert(M, M.fv_idx[b + j]) - c);
    }
    M.fcx[f] = c.x;
    M.fcy[f] = c.y;
    M.fcz[f] = c.z;
    M.Sx[f] = 0.5 * A.x;
    M.Sy[f] = 0.5 * A.y;
    M.Sz[f] = 0.5 * A.z;
    // the owner's and the neighbour's vertex-neighbour lists, so that the staging kernel finds them with
    // one load indexed by the face
    const int o = M.owner[f], nb = M.neigh[f];
    const int ob = M.nb_ptr[o], on = M.nb_ptr[o + 1] - ob;
    const int nbb = nb >= 0 ? M.nb_ptr[nb] : 0, nbn = nb >= 0 ? M.nb_ptr[nb + 1] - nbb : 0;
    M.face_nb[f] = make_int4(ob, on, nbb, nbn);
  }
}

// i-th surface triangle of cell-face entry e (outward for the cell).
__device__ inline void face_triangle(const DevMesh& M, int e, int i, d3& t0, d3& t1, d3& t2) {
  int f = e >= 0 ? e : ~e;
  int b = fv_begin(M, f), k = fv_count(M, f);
  if (k == 3) {
    t0 = vert(M, M.fv_idx[b]);
    t1 = vert(M, M.fv_idx[b + 1]);
    t2 = vert(M, M.fv_idx[b + 2]);
    if (e < 0) {
      d3 t = t1;
      t1 = t2;
      t2 = t;
    }
  } else {
    int j = (i + 1 == k) ? 0 : i + 1;
    t0 = mk3(M.fcx[f], M.fcy[f], M.fcz[f]);
    t1 = vert(M, M.fv_idx[b + i]);
    t2 = vert(M, M.fv_idx[b + j]);
    if (e < 0) {
      d3 t = t1;
      t1 = t2;
      t2 = t;
    }
  }
}

__device__ inline int face_triangle_count(const DevMesh& M, int e) {
  int f = e >= 0 ? e : ~e;
  int k = fv_count(M, f);
  return k == 3 ? 1 : k;
}

// Cell vertex mean (distinct vertices, ascending id), enclosing box, box
// detection, and volume as signed tetrahedra from the vertex mean over the
// surface triangles.  Flags cells that are not closed or not positive.
__global__ void k_cell_geom(DevMesh M) {
  for (int c = grid_stride_start(); c < M.nc; c += grid_stride()) {
    M.flux_near[c] = 1;  // until a reconstruction clears it: no cell is skipped by the update
    M.tag_cell[c] = 0;   // so the first reconstruction clears every plane it does not place
    int vb = M.cv_ptr[c], vn = M.cv_ptr[c + 1] - vb;
    d3 s = mk3(0.0, 0.0, 0.0);
    d3 lo = vert(M, M.cv_idx[vb]), hi = lo;
    for (int i = 0; i < vn; ++i) {
      d3 p = vert(M, M.cv_idx[vb + i]);
      s = s + p;
      lo = vmin(lo, p);
      hi = vmax(hi, p);
    }
    double dn = (double)vn;
    d3 cen = mk3(s.x / dn, s.y / dn, s.z / dn);
    int fb = cf_begin(M, c), fn = cf_count(M, c);
    bool box = vn == 8 && fn == 6;
    if (box) {
      int mask = 0;
      for (int i = 0; i < vn; ++i) {
        d3 p = vert(M, M.cv_idx[vb + i]);
        bool ok = (p.x == lo.x || p.x == hi.x) && (p.y == lo.y || p.y == hi.y) && (p.z == lo.z || p.z == hi.z);
        if (!ok) box = false;
        mask |= 1 << ((p.x == hi.x ? 1 : 0) + (p.y == hi.y ? 2 : 0) + (p.z == hi.z ? 4 : 0));
      }
      if (mask != 255) box = false;
      if (!(lo.x < hi.x && lo.y < hi.y && lo.z < hi.z)) box = false;
      for (int i = 0; i < fn; ++i) {
        int e = M.cf_idx[fb + i];
        int f = e >= 0 ? e : ~e;
        if (fv_count(M, f) != 4) box = false;
      }
    }
    double vol = 0.0, amag = 0.0;
    d3 net = mk3(0.0, 0.0, 0.0);
    for (int i = 0; i < fn; ++i) {
      int e = M.cf_idx[fb + i];
      int f = e >= 0 ? e : ~e;
      double sg = e >= 0 ? 1.0 : -1.0;
      net = net + sg * mk3(M.Sx[f], M.Sy[f], M.Sz[f]);
      amag += fabs(M.Sx[f]) + fabs(M.Sy[f]) + fabs(M.Sz[f]);
      int nt = face_triangle_count(M, e);
      for (int t = 0; t < nt; ++t) {
        d3 t0, t1, t2;
        face_triangle(M, e, t, t0, t1, t2);
        vol += det3f(t0 - cen, t1 - cen, t2 - cen);
      }
    }
    vol *= (1.0 / 6.0);
    M.ccx[c] = cen.x;
    M.ccy[c] = cen.y;
    M.ccz[c] = cen.z;
    M.lox[c] = lo.x;
    M.loy[c] = lo.y;
    M.loz[c] = lo.z;
    M.hix[c] = hi.x;
    M.hiy[c] = hi.y;
    M.hiz[c] = hi.z;
    M.V[c] = vol;
    M.isbox[c] = box ? 1 : 0;
    double nn = fabs(net.x) + fabs(net.y) + fabs(net.z);
    if (!(vol > 0.0) || !(nn <= 1e-12 * amag)) atomicOr(&M.counters[CNT_ERR], ERR_MESH);
  }
}

// ============================================================== tagging and cut-off
// Node value F* = sum w F / sum w over the cells sharing the node (ascending
// cell id), w = 1/|x_v - x_c|^2; node tag in {-1, 0, 1}.
// Counters, fill counters and written-part bounds of one advection step
// (one block).
__device__ inline void reset_advect_state(const DevMesh& M) {
  if (threadIdx.x == 0) {
    M.counters[CNT_FACES] = 0;
    M.counters[CNT_ITEMS] = 0;
    M.counters[CNT_OVER] = 0;
    M.counters[CNT_DEEP] = 0;
    M.counters[CNT_UDEEP] = 0;
  }
  for (int r = threadIdx.x; r < kItemRegions; r += blockDim.x) {
    M.regions[r].item_fill = 0;
    M.regions[r].unit_fill = 0;
    M.regions[r].item_okend = INT_MAX;
    M.regions[r].unit_okend = INT_MAX;
  }
}

constexpr int kNodeCells = 8;

// Node weights of the inverse-distance interpolation, once per mesh: w =
// 1/|x_v - x_c|^2 for every cell of every vertex (list order) and their sum
// per vertex, in the operations and order the node values use them.
__global__ void k_node_weights(DevMesh M) {
  for (int v = grid_stride_start(); v < M.nv; v += grid_stride()) {
    const d3 x = vert(M, v);
    double den = 0.0;
    for (int i = M.vc_ptr[v]; i < M.vc_ptr[v + 1]; ++i) {
      const d3 d = x - cell_centre(M, M.vc_idx[i]);
      const double d2 = (d.x * d.x + d.y * d.y) + d.z * d.z;
      const double w = 1.0 / d2;
      M.vc_w[i] = w;
      den = den + w;
    }
    M.vc_den[v] = den;
  }
}

__global__ void k_node_tag(DevMesh M, const double* __restrict__ F) {
  const double eps = M.eps, one_m = 1.0 - M.eps;
  // the interfacial-cell counter of this reconstruction (first incremented by
  // k_cell_tag, which runs after), and the state of the advection step that
  // follows it (which then needs no reset kernel of its own)
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) M.counters[CNT_CELLS] = 0;
    if (M.lsfir_outer > 0 && threadIdx.x <= kMaxLsfirOuter) M.lsfir_turned[threadIdx.x] = 0;
    reset_advect_state(M);
  }
  for (int v = grid_stride_start(); v < M.nv; v += grid_stride()) {
    if (!vert_live(M, v)) continue;
    const int b = M.vc_ptr[v], n = M.vc_ptr[v + 1] - b;  // n >= 1
    // the first kNodeCells cells' fractions, loads issued together (clamped indices)
    int cq[kNodeCells];
#pragma unroll
    for (int q = 0; q < kNodeCells; ++q) cq[q] = M.vc_idx[b + min(q, n - 1)];
    double fq[kNodeCells];
#pragma unroll
    for (int q = 0; q < kNodeCells; ++q) fq[q] = F[cq[q]];
    bool any = n > kNodeCells;
#pragma unroll
    for (int q = 0; q < kNodeCells; ++q) any = any || (q < n && fq[q] != 0.0);
    // Every fraction 0 (either sign): each product w F is a zero, their sum
    // from +0 is +0, and so is F* = +0 / den, whatever the weights.  Otherwise
    // the weights and their sum (from k_node_weights: the geometry does not
    // change), summed in list order.
    double fs = 0.0;
    if (any) {
      const double den = M.vc_den[v];
      double wq[kNodeCells];
#pragma unroll
      for (int q = 0; q < kNodeCells; ++q) wq[q] = M.vc_w[b + min(q, n - 1)];
      double num = 0.0;
#pragma unroll
      for (int q = 0; q < kNodeCells; ++q) {
        if (q < n) num = num + wq[q] * fq[q];
      }
      for (int i = b + kNodeCells; i < b + n; ++i) num = num + M.vc_w[i] * F[M.vc_idx[i]];
      fs = num / den;
    }
    M.Fstar[v] = fs;
    M.tag_node[v] = fs < eps ? -1 : (fs > one_m ? 1 : 0);
  }
}

// Face tag from its node tags: -1 (all -1), 1 (all 1), else 0.  The step
// derives it where it is used (k_face_sweep); k_face_tag stores it for
// gvof_get_tags.
__device__ inline int8_t face_tag_of(const DevMesh& M, int f) {
  const int b = fv_begin(M, f), n = fv_count(M, f);  // 3 <= n <= kMaxFaceVerts
  int vq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) vq[q] = M.fv_idx[b + min(q, n - 1)];
  int tq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) tq[q] = M.tag_node[vq[q]];  // the first four tags in flight together
  bool allm = true, allp = true;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    allm = allm && tq[q] == -1;
    allp = allp && tq[q] == 1;
  }
  for (int i = b + 4; i < b + n; ++i) {
    int t = M.tag_node[M.fv_idx[i]];
    allm = allm && t == -1;
    allp = allp && t == 1;
  }
  return allm ? -1 : (allp ? 1 : 0);
}

__global__ void k_face_tag(DevMesh M) {
  for (int f = grid_stride_start(); f < M.nf; f += grid_stride()) {
    if (!face_live(M, f)) continue;
    M.tag_face[f] = face_tag_of(M, f);
  }
}

// Cell tag, cut-off of F in place, compaction of the interfacial cells.
__global__ void k_cell_tag(DevMesh M, double* __restrict__ F) {
  const double eps = M.eps, one_m = 1.0 - M.eps;
  int n = M.nc;
  int stride = grid_stride();
  // every thread of a block runs the same number of iterations (block_append holds barriers)
  for (int b = blockIdx.x * blockDim.x; b < n; b += stride) {
    int c = b + threadIdx.x;
    bool inter = false;
    if (c < n && cell_live(M, c)) {
      double f = F[c];
      const int8_t prev = M.tag_cell[c];
      int8_t t = f < eps ? -1 : (f > one_m ? 1 : 0);
      M.tag_cell[c] = t;
      M.flux_near[c] = 0;  // set again by the face sweep for the cells of faces that carry fluid
      if (t == -1) F[c] = 0.0;
      if (t == 1) F[c] = 1.0;
      inter = t == 0;
      // no isosurface until k_iso_local finds one (the ELCIR / CLCIR rings read
      // this flag for every neighbour, interfacial or not)
      if (M.iso_level > 0) M.iso_ok[c] = 0;
      // a plane is placed only in an interfacial cell, so a cell that was not
      // interfacial in the last reconstruction holds a zero plane already
      if (!inter && prev == 0) {
        M.pnx[c] = 0.0;
        M.pny[c] = 0.0;
        M.pnz[c] = 0.0;
        M.pC[c] = 0.0;
      }
    }
    block_append(inter, c, &M.counters[CNT_CELLS], M.list_cells, nullptr);  // counted once by k_recon
  }
}

__device__ inline void insert_sorted(double* a, int& n, double v) {
  int i = n++;
  while (i > 0 && a[i - 1] > v) {
    a[i] = a[i - 1];
    --i;
  }
  a[i] = v;
}

// Solves g(s) = T for s in [s0, s0 + w] where g is the cubic through
// (s0, y0), (s0 + w/3, y1), (s0 + 2w/3, y2), (s0 + w, y3) and decreasing.
__device__ inline double cubic_root(double s0, double w, double y0, double y1, double y2, double y3, double T) {
  double D1 = y1 - y0, D2 = (y2 - 2.0 * y1) + y0, D3 = ((y3 - 3.0 * y2) + 3.0 * y1) - y0;
  double q3 = D3 * (1.0 / 6.0), q2 = 0.5 * D2;
  double ua = 0.0, ub = 3.0;
  double u = (y0 - y3) != 0.0 ? 3.0 * (y0 - T) / (y0 - y3) : 1.5;
  u = fmin(fmax(u, 0.0), 3.0);
  for (int it = 0; it < 64; ++it) {
    // p(u) = y0 + u (D1 + (u-1) (q2 + (u-2) q3))
    double qq = fma(u - 2.0, q3, q2);
    double r = fma(u - 1.0, qq, D1);
    double p = fma(u, r, y0) - T;
    double dr = fma(u - 1.0, q3, qq);
    double dp = fma(u, dr, r);
    if (p > 0.0) ua = u;
    else if (p < 0.0) ub = u;
    else break;
    double un = u - p / dp;
    if (!(un > ua && un < ub)) un = 0.5 * (ua + ub);
    if (fabs(un - u) <= 1e-16 * 3.0) {
      u = un;
      break;
    }
    u = un;
  }
  return fma(u, w * (1.0 / 3.0), s0);
}

// ============================================================== face sweep
// V_d = dt u.S, upwind cell, the flux of faces that need no geometry, and the
// list of faces that need a flux polyhedron.
__global__ void k_face_sweep(DevMesh M, const double* __restrict__ uf, double dt) {
  int n = M.nf;
  int stride = grid_stride();
  // every thread of a block runs the same number of iterations (block_append holds barriers)
  for (int b = blockIdx.x * blockDim.x; b < n; b += stride) {
    int f = b + threadIdx.x;
    bool geo = false;
    if (f < n && face_live(M, f)) {
      // every load before the first store (the compiler cannot move loads
      // above stores through these pointers).  The face's vertex list goes
      // first and is taken alone by the empty asm, so the wait before the
      // node-tag loads it feeds covers only it: the tag chain then overlaps the
      // velocity and area loads (the face tag of face_tag_of, inlined)
      const int fb = fv_begin(M, f), fk = fv_count(M, f);  // 3 <= fk <= kMaxFaceVerts
      int vq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) vq[q] = M.fv_idx[fb + min(q, fk - 1)];
      const d3 u = mk3(uf[f], uf[n + f], uf[2 * n + f]);
      const d3 S = mk3(M.Sx[f], M.Sy[f], M.Sz[f]);
      const int nb = M.neigh[f], ow = M.owner[f];
      asm volatile("" : "+v"(vq[0]), "+v"(vq[1]), "+v"(vq[2]), "+v"(vq[3]));
      int tq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) tq[q] = M.tag_node[vq[q]];
      bool allm = true, allp = true;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        allm = allm && tq[q] == -1;
        allp = allp && tq[q] == 1;
      }
      for (int i = fb + 4; i < fb + fk; ++i) {
        const int tv = M.tag_node[M.fv_idx[i]];
        allm = allm && tv == -1;
        allp = allp && tv == 1;
      }
      const int8_t t = allm ? -1 : (allp ? 1 : 0);
      double vd = face_dt(M, f, dt) * dot_x(u, S);
      M.Vd[f] = vd;
      M.upwind[f] = vd >= 0.0 ? ow : nb;
      if (nb < 0 && vd < 0.0) M.VF[f] = 0.0;
      else if (t == -1) M.VF[f] = 0.0;
      else if (t == 1) M.VF[f] = vd;
      else geo = true;
      if (t != -1) {  // V_F may be nonzero: the update of both cells needs the face sums
        M.flux_near[ow] = 1;
        if (nb >= 0) M.flux_near[nb] = 1;
      }
    }
    block_append(geo, f, &M.counters[CNT_FACES], M.list_faces, nullptr);  // counted once per step by k_flux_sum
  }
}

// ============================================================== flux polyhedra + truncation
constexpr int kFluxLanes = 64;
// Points of a polyhedron, in LDS and in its slot: x_0..x_{I-1}, b_0..b_{I-1},
// apex (2I), face centre (2I+1), then for EMFPA the lateral-face centres
// m_0..m_{I-1} (2I+2..3I+1).
constexpr int kMaxPts = 3 * kMaxFaceVerts + 2;
constexpr int kMaxCand = 2 + 2 * kMaxNeighbours;

// Coverage of a flux polyhedron by the cells its truncation visits (the
// owner, the neighbour and the cells sharing a vertex with either: the
// "several cells" a flux region takes fluid from, Sec. "Fluid advected
// through cell faces").  The polyhedron lies in the convex hull of its points,
// so it stays within those cells when every point lies in one of their
// closed boxes (exactly so on a Cartesian grid, whose candidates' boxes tile
// one box).  Points outside the domain's box need no cell: no fluid is there.
// Bit q of the result: point q of the slot layout lies in [lo, hi].  The
// face's own vertices (q < I) lie in the owner's box and are not tested.
__device__ inline bool in_closed_box(d3 p, d3 lo, d3 hi) {
  return lo.x <= p.x && p.x <= hi.x && lo.y <= p.y && p.y <= hi.y && lo.z <= p.z && p.z <= hi.z;
}
template <class Lds>
__device__ inline d3 slot_point(const Lds& S, int q, int I, d3 c) {
  return q == 2 * I + 1 ? c : mk3(S.px[q], S.py[q], S.pz[q]);
}
template <class Lds>
__device__ inline unsigned cover_bits(const Lds& S, int I, int np, d3 c, d3 lo, d3 hi) {
  unsigned bits = 0;
  for (int q = I; q < np; ++q) bits |= in_closed_box(slot_point(S, q, I, c), lo, hi) ? (1u << q) : 0u;
  return bits;
}
// The points outside the domain's box (the same for every lane).
template <class Lds>
__device__ inline unsigned outside_bits(const DevMesh& M, const Lds& S, int f, int I, int np, d3 c) {
  const double* db = M.dom_box + 6 * problem_of(M, M.face_pid, f);
  return ~cover_bits(S, I, np, c, mk3(db[0], db[1], db[2]), mk3(db[3], db[4], db[5]));
}
// Points of the slot layout that the test covers: 2I + 2 (x, b, apex, face
// centre), and for EMFPA the lateral centres.
__device__ inline int slot_points(int method, int I) { return (method == kEMFPA ? 3 : 2) * I + 2; }
__device__ inline unsigned needed_bits(int I, int np) { return ((np >= 32 ? 0u : (1u << np)) - 1u) & ~((1u << I) - 1u); }

__device__ inline bool sorted_contains(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int v = a[mid];
    if (v == key) return true;
    if (v < key) lo = mid + 1;
    else hi = mid;
  }
  return false;
}

// surface triangle m of cell k (walks the face list when faces are polygons)
__device__ inline void cell_piece(const DevMesh& M, int k, int m, d3& t0, d3& t1, d3& t2) {
  int fb = cf_begin(M, k), fn = cf_count(M, k);
  for (int i = 0; i < fn; ++i) {
    int e = M.cf_idx[fb + i];
    int nt = face_triangle_count(M, e);
    if (m < nt) {
      face_triangle(M, e, m, t0, t1, t2);
      return;
    }
    m -= nt;
  }
  t0 = t1 = t2 = mk3(0.0, 0.0, 0.0);
}

// LDS working set of one wavefront building one flux polyhedron.
struct FluxLds {
  double px[kMaxPts], py[kMaxPts], pz[kMaxPts];  // the polyhedron's points (slot layout)
  double ux[kMaxFaceVerts], uy[kMaxFaceVerts], uz[kMaxFaceVerts];
  double mx[kMaxFaceVerts], my[kMaxFaceVerts], mz[kMaxFaceVerts];
  int cand[kMaxCand];
  int cpre[kMaxCand + 1];
  double clox[kMaxCand], cloy[kMaxCand], cloz[kMaxCand], chix[kMaxCand], chiy[kMaxCand], chiz[kMaxCand];
  double cpnx[kMaxCand], cpny[kMaxCand], cpnz[kMaxCand], cpc[kMaxCand];
  double cccx[kMaxCand], cccy[kMaxCand], cccz[kMaxCand];
  signed char ctag[kMaxCand], cbox[kMaxCand];
};

// Flux polyhedron of face f into S.px/py/pz, in phases over the lanes of the
// face's group (lane = index within the group; the caller puts x_i, u_i of
// the face's vertices in S.px/py/pz[i], S.ux/uy/uz[i] first, and
// synchronises between phases).  FMFPA: lateral planes, back vertices, apex;
// EMFPA: streak-line back vertices, lateral centres, apex.
// Lateral planes: lanes 0..I-1 take the plane through edge i parallel to the
// edge-centre velocity.
template <class Lds>
__device__ inline void poly_lateral(Lds& S, int I, int lane) {
  if (lane < I) {
    int j = (lane + 1 == I) ? 0 : lane + 1;
    d3 ub = mk3(0.5 * (S.ux[lane] + S.ux[j]), 0.5 * (S.uy[lane] + S.uy[j]), 0.5 * (S.uz[lane] + S.uz[j]));
    d3 e = mk3(S.px[j] - S.px[lane], S.py[j] - S.py[lane], S.pz[j] - S.pz[lane]);
    d3 m = cross_x(e, ub);
    S.mx[lane] = m.x;
    S.my[lane] = m.y;
    S.mz[lane] = m.z;
  }
}

// Back vertices: lanes 0..I-1 move x_i back along the line where the two
// lateral planes through x_i meet (or along u_i where they are parallel).
template <class Lds>
__device__ inline void poly_back(const DevMesh& M, Lds& S, int I, double dt, int lane) {
  if (lane < I) {
    int i = lane, ip = (lane == 0) ? I - 1 : lane - 1;
    d3 m0 = mk3(S.mx[ip], S.my[ip], S.mz[ip]), m1 = mk3(S.mx[i], S.my[i], S.mz[i]);
    d3 d = cross_x(m0, m1);
    double dd = dot_x(d, d), q0 = dot_x(m0, m0), q1 = dot_x(m1, m1);
    bool fallback = (q0 == 0.0) || (q1 == 0.0) || (dd <= (M.degen * q0) * q1);
    d3 x = mk3(S.px[i], S.py[i], S.pz[i]), u = mk3(S.ux[i], S.uy[i], S.uz[i]);
    d3 bv;
    if (fallback) bv = x - dt * u;  // back-trace along the streak line
    else {
      double t = dotf(u, d) / dd;  // projection of x - dt u on the line of the two lateral planes
      bv = x - (dt * t) * d;
    }
    S.px[I + i] = bv.x;
    S.py[I + i] = bv.y;
    S.pz[I + i] = bv.z;
  }
}

// EMFPA and NMFPA back vertices: lanes 0..I-1 move x_i back along the
// streak line of Eq. (streak-line2), with the vertex's velocity (EMFPA: the
// value depends on the vertex alone, so every face through it gets the same
// bits) or the face-centre velocity (NMFPA, in S.ux/uy/uz[i] for every i).
// NMFPA keeps b_0 in the apex slot as well: the back face's fan vertex.
template <class Lds>
__device__ inline void poly_streak(Lds& S, int I, double dt, bool nm, int lane) {
  if (lane < I) {
    const double bx = S.px[lane] - dt * S.ux[lane];
    const double by = S.py[lane] - dt * S.uy[lane];
    const double bz = S.pz[lane] - dt * S.uz[lane];
    S.px[I + lane] = bx;
    S.py[I + lane] = by;
    S.pz[I + lane] = bz;
    if (nm && lane == 0) {
      S.px[2 * I] = bx;
      S.py[2 * I] = by;
      S.pz[2 * I] = bz;
    }
  }
}

// EMFPA lateral-face centres: lanes 0..I-1 take the vertex mean of
// (x_i, x_{i+1}, b_{i+1}, b_i), summed in pairs of like points so that the
// faces on either side of the edge get the same bits.
template <class Lds>
__device__ inline void poly_centres(Lds& S, int I, int lane) {
  if (lane < I) {
    const int j = (lane + 1 == I) ? 0 : lane + 1, b = I + lane, bj = I + j, m = 2 * I + 2 + lane;
    S.px[m] = ((S.px[lane] + S.px[j]) + (S.px[b] + S.px[bj])) * 0.25;
    S.py[m] = ((S.py[lane] + S.py[j]) + (S.py[b] + S.py[bj])) * 0.25;
    S.pz[m] = ((S.pz[lane] + S.pz[j]) + (S.pz[b] + S.pz[bj])) * 0.25;
  }
}

// Apex: the back-vertex mean moved along S until the polyhedron's signed
// volume equals V_d (every lane computes the same values; lane 0 stores).
template <class Lds>
__device__ inline void poly_apex(const DevMesh& M, Lds& S, int I, bool em, d3 c, d3 Sv, double vd, int lane) {
  // (FMFPA and EMFPA; NMFPA needs no apex)
  d3 g = mk3(0.0, 0.0, 0.0);
  for (int i = 0; i < I; ++i) g = g + mk3(S.px[I + i], S.py[I + i], S.pz[I + i]);
  double dI = (double)I;
  g = mk3(g.x / dI, g.y / dI, g.z / dI);
  double V0 = 0.0, W = 0.0;
  for (int i = 0; i < I; ++i) {
    int j = (i + 1 == I) ? 0 : i + 1;
    d3 xi = mk3(S.px[i], S.py[i], S.pz[i]) - c, xj = mk3(S.px[j], S.py[j], S.pz[j]) - c;
    d3 bi = mk3(S.px[I + i], S.py[I + i], S.pz[I + i]) - c, bj = mk3(S.px[I + j], S.py[I + j], S.pz[I + j]) - c;
    if (em) {
      const int m = 2 * I + 2 + i;
      const d3 mi = mk3(S.px[m], S.py[m], S.pz[m]) - c;
      V0 += det3f(xj, xi, mi);
      V0 += det3f(xi, bi, mi);
      V0 += det3f(bi, bj, mi);
      V0 += det3f(bj, xj, mi);
      V0 += det3f(g - c, bj, bi);
    } else {
      V0 += det3f(xj, xi, bj) + det3f(xi, bi, bj) + det3f(g - c, bj, bi);
    }
    W += det3f(Sv, bj, bi);
  }
  V0 *= (1.0 / 6.0);
  W *= (1.0 / 6.0);
  double mu = 0.0;
  if (fabs(W) <= 1e-12 * dotf(Sv, Sv)) {
    if (lane == 0) atomicOr(&M.counters[CNT_ERR], ERR_APEX);
  } else {
    mu = (vd - V0) / W;
  }
  if (lane == 0) {
    S.px[2 * I] = fma(mu, Sv.x, g.x);
    S.py[2 * I] = fma(mu, Sv.y, g.y);
    S.pz[2 * I] = fma(mu, Sv.z, g.z);
  }
}

// Bounding box of the polyhedron (the face centre included; an EMFPA lateral
// centre, a rounded mean of four points already in the box, cannot leave it:
// rounding is monotone).
template <class Lds>
__device__ inline void poly_box(const Lds& S, int I, d3 c, d3& plo, d3& phi) {
  plo = c;
  phi = c;
  for (int i = 0; i <= 2 * I; ++i) {
    d3 p = mk3(S.px[i], S.py[i], S.pz[i]);
    plo = vmin(plo, p);
    phi = vmax(phi, p);
  }
}

// The whole polyhedron of face f with block barriers between the phases.
// Returns the face centre, area vector and the polyhedron's bounding box.
template <class Lds>
__device__ inline void flux_polyhedron(const DevMesh& M, Lds& S, int f, int b0, int I,
                                       const double* __restrict__ vel, double dt, d3& c, d3& Sv, d3& plo, d3& phi) {
  const int lane = threadIdx.x;
  const bool nm = M.method == kNMFPA;
  const int vs = nm ? M.nf : M.nv;  // vel: face velocities (NMFPA) or vertex velocities
  if (lane < I) {
    int v = M.fv_idx[b0 + lane];
    const int vi = nm ? f : v;
    S.px[lane] = M.vx[v];
    S.py[lane] = M.vy[v];
    S.pz[lane] = M.vz[v];
    S.ux[lane] = vel[vi];
    S.uy[lane] = vel[vs + vi];
    S.uz[lane] = vel[2 * vs + vi];
  }
  __syncthreads();
  if (M.method != kFMFPA) {
    poly_streak(S, I, dt, nm, lane);
    __syncthreads();
    if (!nm) poly_centres(S, I, lane);
  } else {
    poly_lateral(S, I, lane);
    __syncthreads();
    poly_back(M, S, I, dt, lane);
  }
  __syncthreads();
  c = mk3(M.fcx[f], M.fcy[f], M.fcz[f]);
  Sv = mk3(M.Sx[f], M.Sy[f], M.Sz[f]);
  if (!nm) poly_apex(M, S, I, M.method == kEMFPA, c, Sv, M.Vd[f], lane);
  __syncthreads();
  poly_box(S, I, c, plo, phi);
}

// Candidate cells of face f (owner, neighbour and every cell sharing a vertex
// with either) that hold fluid and whose boxes meet the polyhedron's box,
// cached in LDS in a fixed order; cpre holds the prefix of pieces per
// candidate (1 for a box, one per surface triangle otherwise).
__device__ inline int flux_candidates(const DevMesh& M, FluxLds& S, int f, d3 plo, d3 phi) {
  const int lane = threadIdx.x;
  const int o = M.owner[f], nbr = M.neigh[f];
  const int ob = M.nb_ptr[o], on = M.nb_ptr[o + 1] - ob;
  const int nbb = nbr >= 0 ? M.nb_ptr[nbr] : 0, nbn = nbr >= 0 ? M.nb_ptr[nbr + 1] - nbb : 0;
  const int L = 1 + on + (nbr >= 0 ? 1 + nbn : 0);
  int ncand = 0;
  for (int j0 = 0; j0 < L; j0 += kFluxLanes) {
    int j = j0 + lane;
    bool keep = false;
    int k = -1;
    int8_t tg = -1;
    d3 klo = mk3(0, 0, 0), khi = klo;
    if (j < L) {
      bool second = j > on;
      if (j == 0) k = o;
      else if (j <= on) k = M.nb_idx[ob + j - 1];
      else if (j == on + 1) k = nbr;
      else k = M.nb_idx[nbb + j - on - 2];
      tg = M.tag_cell[k];
      keep = tg != -1;
      if (keep && second) keep = !(k == o || sorted_contains(M.nb_idx + ob, on, k));
      if (keep) {
        klo = mk3(M.lox[k], M.loy[k], M.loz[k]);
        khi = mk3(M.hix[k], M.hiy[k], M.hiz[k]);
        keep = box_overlap(plo, phi, klo, khi);
      }
    }
    unsigned long long bm = __ballot(keep);
    if (keep) {
      int pos = ncand + __popcll(bm & ((1ull << lane) - 1ull));
      S.cand[pos] = k;
      S.clox[pos] = klo.x; S.cloy[pos] = klo.y; S.cloz[pos] = klo.z;
      S.chix[pos] = khi.x; S.chiy[pos] = khi.y; S.chiz[pos] = khi.z;
      S.ctag[pos] = tg;
      S.cpnx[pos] = M.pnx[k]; S.cpny[pos] = M.pny[k]; S.cpnz[pos] = M.pnz[k]; S.cpc[pos] = M.pC[k];
      S.cccx[pos] = M.ccx[k]; S.cccy[pos] = M.ccy[k]; S.cccz[pos] = M.ccz[k];
      int box = M.isbox[k];
      S.cbox[pos] = (signed char)box;
      int np = 1;
      if (!box) {
        np = 0;
        for (int q = cf_begin(M, k); q < cf_begin(M, k) + cf_count(M, k); ++q) np += face_triangle_count(M, M.cf_idx[q]);
      }
      S.cpre[pos + 1] = np;
    }
    ncand += __popcll(bm);
  }
  __syncthreads();
  if (lane == 0) {
    S.cpre[0] = 0;
    for (int kc = 0; kc < ncand; ++kc) S.cpre[kc + 1] += S.cpre[kc];
  }
  __syncthreads();
  return ncand;
}

// vol(cell k ∩ T [∩ PLIC half-space]) for a non-box cell: signed sum over the
// cell's surface tetrahedra.  With DEEP false, a piece cut by more than
// kMaxRegCuts planes makes the call return false (the caller defers the pair).
template <bool DEEP>
__device__ __attribute__((always_inline)) inline bool tet_cell_pieces_volume(const DevMesh& M, int k, d3 cc, const Tet& T, const Leaf& leaf,
                                              double& out) {
  d3 tlo = vmin(vmin(T.p0, T.p1), vmin(T.p2, T.p3)), thi = vmax(vmax(T.p0, T.p1), vmax(T.p2, T.p3));
  double acc = 0.0;
  const TetCont Tc = tet_container(T.p0, T.p1, T.p2, T.p3);
  double sc[4];
  apex_dists(Tc, cc, sc);
  int fb = cf_begin(M, k), fn = cf_count(M, k);
  for (int i = 0; i < fn; ++i) {
    int e = M.cf_idx[fb + i];
    int nt = face_triangle_count(M, e);
    for (int q = 0; q < nt; ++q) {
      d3 t0, t1, t2;
      face_triangle(M, e, q, t0, t1, t2);
      unsigned w;
      if (!unit_rule(T, tlo, thi, Tc, sc, cc, t0, t1, t2, w)) continue;
      const double s6 = det3f(t0 - cc, t1 - cc, t2 - cc);
      Tet X;
      TetCont C;
      unit_clip_value_setup(T, cc, t0, t1, t2, w, X, C);
      double v = clip_masked_tet(X, C, w & 15u, leaf);
      acc += s6 > 0.0 ? v : -v;
    }
  }
  out = acc;
  return true;
}

// LDS of the staging kernel, per face: the polyhedron, the owner's neighbour
// list and up to kPrepCand candidate cells (first staged as listed, then
// compacted in place to those that survive the tests).
constexpr int kPrepCand = 64;
struct PrepLds {
  double px[kMaxPts], py[kMaxPts], pz[kMaxPts];
  double ux[kMaxFaceVerts], uy[kMaxFaceVerts], uz[kMaxFaceVerts];
  double mx[kMaxFaceVerts], my[kMaxFaceVerts], mz[kMaxFaceVerts];
  int onb[kMaxNeighbours];
  int cand[kPrepCand];
  double clox[kPrepCand], cloy[kPrepCand], cloz[kPrepCand], chix[kPrepCand], chiy[kPrepCand], chiz[kPrepCand];
  signed char cbox[kPrepCand], ctag[kPrepCand];
};

// Hands LDS data between the lanes of a wavefront: the wavefront's LDS
// operations complete in order, so waiting for its own is enough; its global
// loads stay in flight, and the compiler moves no memory access across the
// wait.  (Blocks of the staging kernels are one wavefront.)
__device__ inline void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Candidate j of a face: the owner, the owner's neighbours, the neighbour,
// then the neighbour's neighbours.
__device__ inline int candidate_cell(const DevMesh& M, int j, int o, int ob, int on, int nbr, int nbb) {
  if (j == 0) return o;
  if (j <= on) return M.nb_idx[ob + j - 1];
  if (j == on + 1) return nbr;
  return M.nb_idx[nbb + j - on - 2];
}

// Pair word tm: bits 0-5 the flux tet (< 5 kMaxFaceVerts), 6-11 the mask of
// the box planes that cut it, bit 12 set when the first of those cuts keeps
// three tetrahedra, 13-15 the face's vertex count minus 3.
constexpr int kTmWideBit = 12;
static_assert(5 * kMaxFaceVerts <= 64 && kMaxFaceVerts - 3 <= 7, "pair word fields");
__device__ inline unsigned tm_tet(unsigned tm) { return tm & 63u; }
__device__ inline unsigned tm_mask(unsigned tm) { return (tm >> 6) & 63u; }
__device__ inline int tm_verts(unsigned tm) { return (int)((tm >> 13) & 7u) + 3; }
__device__ inline unsigned tm_word(int t, unsigned mask, int I) {
  return (unsigned)t | (mask << 6) | ((unsigned)(I - 3) << 13);
}

// Test of staged candidate kc against flux tet t: the tet's box meets the
// cell's box and, for a box cell, the tet is not entirely outside one box
// plane.
__device__ inline bool pair_test(const PrepLds& S, d3 c, int I, int method, int TF, int q, unsigned& tm, int& kc) {
  const int t = q % TF;
  kc = q / TF;
  int i1, i2, i3;
  flux_tet_points(t, I, method, i1, i2, i3);
  Tet T{c, mk3(S.px[i1], S.py[i1], S.pz[i1]), mk3(S.px[i2], S.py[i2], S.pz[i2]), mk3(S.px[i3], S.py[i3], S.pz[i3])};
  d3 tlo = vmin(vmin(T.p0, T.p1), vmin(T.p2, T.p3)), thi = vmax(vmax(T.p0, T.p1), vmax(T.p2, T.p3));
  BoxCont B{mk3(S.clox[kc], S.cloy[kc], S.cloz[kc]), mk3(S.chix[kc], S.chiy[kc], S.chiz[kc])};
  const bool keep = box_overlap(tlo, thi, B.lo, B.hi);
  const unsigned mask = keep && S.cbox[kc] ? box_cut_mask(tlo, thi, B) : 0u;
  tm = tm_word(t, mask, I);
  if (mask) {
    // the first cut keeps three tetrahedra (two or more vertices inside) or one:
    // a hint for grouping pairs of like work in the truncation kernel.  Inside
    // plane 2a means x_a > lo_a, inside plane 2a+1 means x_a < hi_a (the sign
    // of the plane's distance, as in box_cut_mask).
    const int l = __builtin_ctz(mask), a = l >> 1;
    const bool up = (l & 1) != 0;
    const double bound = a == 0 ? (up ? B.hi.x : B.lo.x) : (a == 1 ? (up ? B.hi.y : B.lo.y) : (up ? B.hi.z : B.lo.z));
    const double c0 = a == 0 ? T.p0.x : (a == 1 ? T.p0.y : T.p0.z), c1 = a == 0 ? T.p1.x : (a == 1 ? T.p1.y : T.p1.z);
    const double c2 = a == 0 ? T.p2.x : (a == 1 ? T.p2.y : T.p2.z), c3 = a == 0 ? T.p3.x : (a == 1 ? T.p3.y : T.p3.z);
    const int inside = up ? (c0 < bound) + (c1 < bound) + (c2 < bound) + (c3 < bound)
                          : (c0 > bound) + (c1 > bound) + (c2 > bound) + (c3 > bound);
    tm |= (inside >= 2 ? 1u : 0u) << kTmWideBit;
  }
  return keep;
}

// Reserves count pairs for face slot it in region it % kItemRegions of the
// pair buffer.  Returns the first index, or -1 when the region is full: the
// face then goes to the overflow kernel.
__device__ inline int reserve_pairs(const DevMesh& M, int it, int f, int count) {
  const int r = it % kItemRegions;
  const int rsize = M.item_cap / kItemRegions;
  int base = atomicAdd(&M.regions[r].item_fill, count);
  if (base + count > rsize) {
    // every reservation before this one in atomic order fitted and every
    // later one fails: the region's written part is [0, smallest failed base)
    atomicMin(&M.regions[r].item_okend, base);
    M.item_cnt[it] = -1;
    M.list_over[atomicAdd(&M.counters[CNT_OVER], 1)] = f;
    return -1;
  }
  base += r * rsize;
  M.item_off[it] = base;
  M.item_cnt[it] = count;
  return base;
}

__device__ inline void write_pair(const DevMesh& M, int i, int it, int cell, unsigned tm) {
  M.item_slot[i] = it;
  M.item_cell[i] = cell;
  M.item_tm[i] = (unsigned short)tm;
}

// Stage the flux work of every listed face, a group of G lanes per face
// (64 / G faces per wavefront): build its flux polyhedron (stored per slot),
// gather the candidate cells that hold fluid and whose boxes meet the
// polyhedron's box, then emit one (face, cell, flux tet) pair for every flux
// tet whose box meets such a cell's box (box cells: the tet is also not
// entirely outside one box plane, and the pair carries the mask of the box
// planes that cut it).  Pairs of one face are contiguous and in a fixed
// order.  Faces with more than kPrepCand such cells or without room in the
// staging buffers go to the overflow kernel.
// The loads of the face's vertices and of its first 64 listed cells form two
// independent chains; they are issued together, straight-line with clamped
// indices, and the cells' data go to LDS as soon as they arrive.
// METHOD is the mesh's flux polyhedron method (an instance per method keeps
// each instance's registers to its own path); vel holds the vertex
// velocities (FMFPA, EMFPA) or the face velocities (NMFPA).
template <int G, int METHOD>
__global__ __launch_bounds__(kFluxLanes, 4) void k_flux_prep(DevMesh M, const double* __restrict__ vel, double dt) {
  static_assert(G == 32 || G == 64, "lanes per face");
  constexpr int NG = kFluxLanes / G;  // faces per wavefront
  constexpr int NR = kFluxLanes / G;  // rounds of G lanes over the first 64 listed cells
  __shared__ PrepLds SS[NG];
  const int lane = threadIdx.x;
  const int grp = lane / G, sub = lane - grp * G, gbase = grp * G;
  PrepLds& S = SS[grp];
  const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
  const unsigned long long lbelow = ((1ull << lane) - 1ull) & gmask;
  const int nfaces = M.counters[CNT_FACES];
  const int nv = M.nv;
  for (int it = blockIdx.x * NG + grp; it < nfaces; it += gridDim.x * NG) {
    const int f = M.list_faces[it];
    if (it >= M.poly_cap) {
      if (sub == 0) M.list_over[atomicAdd(&M.counters[CNT_OVER], 1)] = f;
      continue;
    }
    // Loads first, straight-line with clamped indices (every lane reads valid
    // memory), so both chains are in flight together.
    const int b0 = fv_begin(M, f), I = fv_count(M, f);
    const int o = M.owner[f], nbr = M.neigh[f];
    const d3 c = mk3(M.fcx[f], M.fcy[f], M.fcz[f]);
    const d3 Sv = mk3(M.Sx[f], M.Sy[f], M.Sz[f]);
    const double vd = M.Vd[f];
    const int4 fnb = M.face_nb[f];
    const int ob = fnb.x, on = fnb.y, nbb = fnb.z, nbn = fnb.w;
    // the face's problem: its step (face_dt) and its domain's box (for the coverage test), loaded here with
    // the face's other data rather than behind the polyhedron's LDS phases
    const int pid = problem_of(M, M.face_pid, f);
    const double fdt = M.prob_dt ? M.prob_dt[pid] : dt;
    const double* db = M.dom_box + 6 * pid;
    const d3 dlo = mk3(db[0], db[1], db[2]), dhi = mk3(db[3], db[4], db[5]);
    const int L = 1 + on + (nbr >= 0 ? 1 + nbn : 0);
    // listed cells j = sub + G r (r < NR); lanes past the list read the owner
    int kq[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int j = sub + G * r;
      const bool in_list = j < L;
      const bool listed = in_list & (j != 0) & (j != on + 1);
      int idx = j <= on ? ob + j - 1 : nbb + j - on - 2;
      idx = listed ? idx : 0;
      const int kl = M.nb_idx[idx];
      int k = listed ? kl : o;
      kq[r] = (in_list & (j == on + 1)) ? nbr : k;
    }
    const int v = M.fv_idx[b0 + min(sub, I - 1)];
    const d3 x = vert(M, v);
    // the vertex's velocity, or for NMFPA the face's (one for all vertices)
    const int vi = METHOD == kNMFPA ? f : v, vs = METHOD == kNMFPA ? M.nf : nv;
    const d3 u = mk3(vel[vi], vel[vs + vi], vel[2 * vs + vi]);
    int8_t tq[NR];
    signed char bq[NR];
    d3 loq[NR], hiq[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int k = kq[r];
      tq[r] = M.tag_cell[k];
      loq[r] = mk3(M.lox[k], M.loy[k], M.loz[k]);
      hiq[r] = mk3(M.hix[k], M.hiy[k], M.hiz[k]);
      bq[r] = M.isbox[k];
    }
    // then the LDS hand-offs: the face's vertices, the owner's list and the listed cells
    if (sub < I) {
      S.px[sub] = x.x; S.py[sub] = x.y; S.pz[sub] = x.z;
      S.ux[sub] = u.x; S.uy[sub] = u.y; S.uz[sub] = u.z;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int j = sub + G * r;
      if (j >= 1 && j <= on) S.onb[j - 1] = kq[r];
      S.cand[j] = kq[r];
      S.ctag[j] = tq[r];
      S.clox[j] = loq[r].x; S.cloy[j] = loq[r].y; S.cloz[j] = loq[r].z;
      S.chix[j] = hiq[r].x; S.chiy[j] = hiq[r].y; S.chiz[j] = hiq[r].z;
      S.cbox[j] = bq[r];
    }
    constexpr bool em = METHOD == kEMFPA, nm = METHOD == kNMFPA;
    if (em || nm) {  // the lane holding x_i, u_i moves it back (EMFPA: then the centres)
      if (sub < I) {
        const d3 b = mk3(x.x - fdt * u.x, x.y - fdt * u.y, x.z - fdt * u.z);
        S.px[I + sub] = b.x;
        S.py[I + sub] = b.y;
        S.pz[I + sub] = b.z;
        if (nm && sub == 0) {  // b_0 also in the apex slot: the back face's fan vertex
          S.px[2 * I] = b.x;
          S.py[2 * I] = b.y;
          S.pz[2 * I] = b.z;
        }
      }
      wave_lds_sync();
      if (em) poly_centres(S, I, sub);
    } else {
      wave_lds_sync();
      poly_lateral(S, I, sub);
      wave_lds_sync();
      poly_back(M, S, I, fdt, sub);
    }
    wave_lds_sync();
    if (!nm) {  // NMFPA's prism has the volume V_d as it is
      poly_apex(M, S, I, em, c, Sv, vd, sub);
      wave_lds_sync();
    }
    d3 plo, phi;
    poly_box(S, I, c, plo, phi);
    // coverage: every point of the polyhedron in the box of a listed cell, or outside the domain's box
    // (lanes past the list hold the owner, itself listed).  The first G listed cells (the owner, its
    // neighbours, ...) nearly always hold every point, so the other cells and the domain's box are tested
    // only when a point is left over: the same flag, for a fraction of the tests.
    const int npt = slot_points(METHOD, I);
    const unsigned need = needed_bits(I, npt);
    unsigned cov = cover_bits(S, I, npt, c, mk3(S.clox[sub], S.cloy[sub], S.cloz[sub]),
                              mk3(S.chix[sub], S.chiy[sub], S.chiz[sub]));
#pragma unroll
    for (int o2 = 1; o2 < G; o2 <<= 1) cov |= __shfl_xor(cov, o2);
    const bool covered = (cov & need) == need;  // uniform over the group
    if (!covered) {
#pragma unroll
      for (int r = 1; r < NR; ++r) {
        const int j = sub + G * r;
        cov |= cover_bits(S, I, npt, c, mk3(S.clox[j], S.cloy[j], S.cloz[j]), mk3(S.chix[j], S.chiy[j], S.chiz[j]));
      }
      cov |= ~cover_bits(S, I, npt, c, dlo, dhi);  // points outside the domain's box need no cell
    }
    double* P = M.poly + (size_t)it * M.pts_per_slot * 3;
    // the points, the face centre (the flux tets' common vertex), the lateral centres
    if (sub <= 2 * I || (em && sub >= 2 * I + 2 && sub <= 3 * I + 1)) {
      P[3 * sub] = S.px[sub];
      P[3 * sub + 1] = S.py[sub];
      P[3 * sub + 2] = S.pz[sub];
    } else if (sub == 2 * I + 1) {
      P[3 * sub] = c.x;
      P[3 * sub + 1] = c.y;
      P[3 * sub + 2] = c.z;
    }
    // candidates: cells that hold fluid, not listed before (a cell of the
    // neighbour's list that is the owner or on the owner's list) and whose
    // boxes meet the polyhedron's; compacted in place (a cell moves only to
    // a slot already read)
    int ncand = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int j = sub + G * r;
      const int k = S.cand[j];
      const d3 klo = mk3(S.clox[j], S.cloy[j], S.cloz[j]), khi = mk3(S.chix[j], S.chiy[j], S.chiz[j]);
      const signed char kb = S.cbox[j];
      bool keep = j < L && S.ctag[j] != -1;
      if (keep && j > on) keep = !(k == o || sorted_contains(S.onb, on, k));
      keep = keep && box_overlap(plo, phi, klo, khi);
      const unsigned long long bm = __ballot(keep) & gmask;
      wave_lds_sync();  // every lane has read its slot before any slot is rewritten
      if (keep) {
        const int pos = ncand + __popcll(bm & lbelow);
        S.cand[pos] = k;
        S.clox[pos] = klo.x; S.cloy[pos] = klo.y; S.cloz[pos] = klo.z;
        S.chix[pos] = khi.x; S.chiy[pos] = khi.y; S.chiz[pos] = khi.z;
        S.cbox[pos] = kb;
      }
      ncand += __popcll(bm);
    }
    for (int j0 = kFluxLanes; j0 < L; j0 += G) {  // more than 64 cells listed (general meshes only)
      const int j = j0 + sub;
      bool keep = false;
      int k = o;
      d3 klo = mk3(0.0, 0.0, 0.0), khi = klo;
      signed char kb = 0;
      if (j < L) {
        k = candidate_cell(M, j, o, ob, on, nbr, nbb);
        klo = mk3(M.lox[k], M.loy[k], M.loz[k]);
        khi = mk3(M.hix[k], M.hiy[k], M.hiz[k]);
        if (!covered) cov |= cover_bits(S, I, npt, c, klo, khi);  // the coverage test, if a point is left
        keep = M.tag_cell[k] != -1 && !(k == o || sorted_contains(S.onb, on, k));
        if (keep) {
          kb = M.isbox[k];
          keep = box_overlap(plo, phi, klo, khi);
        }
      }
      const unsigned long long bm = __ballot(keep) & gmask;
      if (keep) {
        const int pos = ncand + __popcll(bm & lbelow);
        if (pos < kPrepCand) {
          S.cand[pos] = k;
          S.clox[pos] = klo.x; S.cloy[pos] = klo.y; S.cloz[pos] = klo.z;
          S.chix[pos] = khi.x; S.chiy[pos] = khi.y; S.chiz[pos] = khi.z;
          S.cbox[pos] = kb;
        }
      }
      ncand += __popcll(bm);
    }
    if (!covered) {
#pragma unroll
      for (int o2 = 1; o2 < G; o2 <<= 1) cov |= __shfl_xor(cov, o2);
      if (sub == 0 && (cov & need) != need) atomicOr(&M.counters[CNT_ERR], ERR_COVER);
    }
    wave_lds_sync();
    if (ncand > kPrepCand) {
      if (sub == 0) {
        M.item_cnt[it] = -1;
        M.list_over[atomicAdd(&M.counters[CNT_OVER], 1)] = f;
      }
      continue;
    }
    const int TF = flux_tet_count(METHOD, I);
    const int total = ncand * TF;
    if (total <= kFluxLanes) {
      // up to NR rounds: the tests stay in registers between counting and writing
      bool kp[NR];
      unsigned tmq[NR];
      int kcq[NR];
      unsigned long long bmq[NR];
      int count = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int q = sub + G * r;
        tmq[r] = 0;
        kcq[r] = 0;
        kp[r] = q < total && pair_test(S, c, I, METHOD, TF, q, tmq[r], kcq[r]);
        bmq[r] = __ballot(kp[r]) & gmask;
        count += __popcll(bmq[r]);
      }
      int base = 0;
      if (sub == 0) base = reserve_pairs(M, it, f, count);
      base = __shfl(base, gbase);
      if (base >= 0) {
        int written = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (kp[r]) write_pair(M, base + written + __popcll(bmq[r] & lbelow), it, S.cand[kcq[r]], tmq[r]);
          written += __popcll(bmq[r]);
        }
      }
    } else {
      // pass 0 counts, pass 1 writes into the reserved range
      int count = 0;
      for (int q0 = 0; q0 < total; q0 += G) {
        unsigned tm;
        int kc;
        const bool kp = q0 + sub < total && pair_test(S, c, I, METHOD, TF, q0 + sub, tm, kc);
        count += __popcll(__ballot(kp) & gmask);
      }
      int base = 0;
      if (sub == 0) base = reserve_pairs(M, it, f, count);
      base = __shfl(base, gbase);
      if (base >= 0) {
        int written = 0;
        for (int q0 = 0; q0 < total; q0 += G) {
          unsigned tm = 0;
          int kc = 0;
          const bool kp = q0 + sub < total && pair_test(S, c, I, METHOD, TF, q0 + sub, tm, kc);
          const unsigned long long bm = __ballot(kp) & gmask;
          if (kp) write_pair(M, base + written + __popcll(bm & lbelow), it, S.cand[kc], tm);
          written += __popcll(bm);
        }
      }
    }
    wave_lds_sync();
  }
}

// One lane per staged pair: signed fluid volume of (flux tet ∩ cell).  Two
// instances, one for box cells and one for general cells, each skipping the
// other kind, so each carries only its own registers.
// Flux tet of a staged pair from its pair word alone: the tet and the face's
// vertex count are in the word, the points and the face centre in the slot.
__device__ inline Tet staged_tet(const DevMesh& M, int slot, unsigned tm) {
  const int t = tm_tet(tm), I = tm_verts(tm);
  const double* P = M.poly + (size_t)slot * M.pts_per_slot * 3;
  int i1, i2, i3;
  flux_tet_points(t, I, M.method, i1, i2, i3);
  const int ic = 2 * I + 1;
  return Tet{mk3(P[3 * ic], P[3 * ic + 1], P[3 * ic + 2]), mk3(P[3 * i1], P[3 * i1 + 1], P[3 * i1 + 2]),
             mk3(P[3 * i2], P[3 * i2 + 1], P[3 * i2 + 2]), mk3(P[3 * i3], P[3 * i3 + 1], P[3 * i3 + 2])};
}

// Pair buffer regions: block b serves region b % kItemRegions and strides over
// that region's filled part with the other gridDim.x / kItemRegions blocks of
// the same region (the grid is a multiple of kItemRegions).
__device__ inline int region_blocks() { return gridDim.x / kItemRegions; }
// Written pairs of region r: reservations that did not fit leave the fill
// counter past what was written, so the count stops at the first of them.
__device__ inline int region_items(const DevMesh& M, int r, int rsize) {
  return min(min(M.regions[r].item_fill, M.regions[r].item_okend), rsize);
}

// Box-cell pairs, one lane per pair.  A pair's work grows with the number of
// box planes cutting its tetrahedron (up to 9 leaves for two), with the
// children of the first cut (one or three) and with whether the cell's
// interface cuts the leaves, and a wavefront runs as long as its slowest
// lane (and runs every path one of its lanes takes), so each block first
// ranks its pairs by that work in LDS (a counting sort, most work first)
// and each thread then clips the pair at its rank: most wavefronts see pairs
// of one kind.  Each pair's volume goes to its own slot, so the order changes
// no result.  A block pass ranks 1024 pairs: where general-cell pairs share
// the buffer (a batch of problems on both kinds of grid) only the box pairs
// among them are clipped, and fewer would leave most lanes of the clip idle.
constexpr int kItemsBlock = 256;
constexpr int kItemsPerThread = 4;  // pairs ranked together per block: kItemsBlock x this
__global__ __launch_bounds__(kItemsBlock) void k_flux_items_box(DevMesh M) {
  constexpr int CHUNK = kItemsBlock * kItemsPerThread;
  constexpr int VW = CHUNK / 64;  // the chunk as wavefront-sized runs ("virtual wavefronts")
  __shared__ int s_list[CHUNK], s_cell[CHUNK], s_slot[CHUNK];
  __shared__ unsigned short s_tm[CHUNK];
  // classes: 2 x (none; then per cut count, first cut keeping one or three),
  // the factor 2 for cells cut by their interface (the leaves then take the
  // half-space fraction) or not
  constexpr int NCLS = 2 * (2 * kMaxRegCuts + 1);
  __shared__ int s_off[VW][NCLS];
  __shared__ int s_n;
  const int rsize = M.item_cap / kItemRegions;
  const int r = blockIdx.x % kItemRegions, sub = blockIdx.x / kItemRegions;
  const int fill = region_items(M, r, rsize);
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  // every thread of a block makes the same number of passes (block barriers)
  for (int b = sub * CHUNK; b < fill; b += region_blocks() * CHUNK) {
    // each thread classifies kItemsPerThread pairs, b + threadIdx.x + h kItemsBlock
    int cls[kItemsPerThread], idx[kItemsPerThread], kc[kItemsPerThread], sl[kItemsPerThread];
    unsigned tmh[kItemsPerThread];
    unsigned long long mh[kItemsPerThread];
#pragma unroll
    for (int h = 0; h < kItemsPerThread; ++h) {
      const int li = b + threadIdx.x + h * kItemsBlock;
      int c = -1;  // work class (more work, higher), or -1: nothing for the register clip
      const int i = r * rsize + li;
      int k = 0, slot = 0;
      unsigned tm = 0;
      if (li < fill) {
        k = M.item_cell[i];
        tm = M.item_tm[i];
        slot = M.item_slot[i];
        const int8_t tg = M.tag_cell[k];
        if (M.isbox[k]) {
          const int nc = cut_count(tm_mask(tm));
          if (nc > kMaxRegCuts) M.list_deep[atomicAdd(&M.counters[CNT_DEEP], 1)] = i;  // deferred (rare)
          else c = 2 * (nc == 0 ? 0 : 2 * nc - 1 + (int)((tm >> kTmWideBit) & 1u)) + (tg == 0 ? 1 : 0);
        }
      }
      unsigned long long m = 0;
#pragma unroll
      for (int q = 0; q < NCLS; ++q) {
        const unsigned long long bq = __ballot(c == q);
        if (lane == 0) s_off[h * (kItemsBlock / 64) + w][q] = __popcll(bq);
        m = c == q ? bq : m;
      }
      cls[h] = c;
      idx[h] = i;
      kc[h] = k;
      sl[h] = slot;
      tmh[h] = tm;
      mh[h] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int c = NCLS - 1; c >= 0; --c)
        for (int v = 0; v < VW; ++v) {
          const int n = s_off[v][c];
          s_off[v][c] = t;
          t += n;
        }
      s_n = t;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < kItemsPerThread; ++h) {
      if (cls[h] >= 0) {
        const int pos = s_off[h * (kItemsBlock / 64) + w][cls[h]] + __popcll(mh[h] & below);
        s_list[pos] = idx[h];  // the pair and what the clip needs of it first
        s_cell[pos] = kc[h];
        s_slot[pos] = sl[h];
        s_tm[pos] = (unsigned short)tmh[h];
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < s_n; q += kItemsBlock) {  // ranks in order of work, most first
      const int ip = s_list[q];
      const int k = s_cell[q];
      const unsigned tm = s_tm[q];
      const Tet T = staged_tet(M, s_slot[q], tm);
      const double sT = tet6(T);
      double v = 0.0;
      if (sT != 0.0) {
        Leaf leaf;
        leaf.useH = M.tag_cell[k] == 0;
        leaf.hn = mk3(M.pnx[k], M.pny[k], M.pnz[k]);
        leaf.hd = M.pC[k];
        BoxCont B{mk3(M.lox[k], M.loy[k], M.loz[k]), mk3(M.hix[k], M.hiy[k], M.hiz[k])};
        v = clip_masked(T, B, tm_mask(tm), leaf);
        if (sT < 0.0) v = -v;
      }
      M.item_vol[ip] = v;
    }
    __syncthreads();  // s_list and s_off are reused by the next pass
  }
}

// Surface tetrahedron p of cell k: (vertex mean, outward triangle), with its
// orientation sign.
__device__ inline void cell_sigma(const DevMesh& M, int k, int p, bool tri_only, d3& t0, d3& t1, d3& t2) {
  if (tri_only) {
    const int o = M.tri_off[k];
    if (M.tri_off[k + 1] > o) {  // cached at bind: one contiguous read instead of a chain of gathers
      const double* q = M.tri_xyz + 9 * (size_t)(o + p);
      t0 = mk3(q[0], q[1], q[2]);
      t1 = mk3(q[3], q[4], q[5]);
      t2 = mk3(q[6], q[7], q[8]);
    } else {
      face_triangle(M, M.cf_idx[cf_begin(M, k) + p], 0, t0, t1, t2);
    }
  } else {
    cell_piece(M, k, p, t0, t1, t2);
  }
}

// Fills the surface-triangle cache (bind time).
__global__ void k_tri_cache(DevMesh M) {
  for (int c = grid_stride_start(); c < M.nc; c += grid_stride()) {
    const int o = M.tri_off[c], n = M.tri_off[c + 1] - o;
    for (int p = 0; p < n; ++p) {
      d3 t0, t1, t2;
      face_triangle(M, M.cf_idx[cf_begin(M, c) + p], 0, t0, t1, t2);
      double* q = M.tri_xyz + 9 * (size_t)(o + p);
      q[0] = t0.x; q[1] = t0.y; q[2] = t0.z;
      q[3] = t1.x; q[4] = t1.y; q[5] = t1.z;
      q[6] = t2.x; q[7] = t2.y; q[8] = t2.z;
    }
  }
}

__device__ inline int cell_piece_count(const DevMesh& M, int k) { return M.cell_np[k]; }

// Pairs with a general (non-box) cell, stage 1: a group of LPP lanes per pair
// (8, 16, 32 or 64; the lane-to-pair mapping is a launch choice), lane j of the
// group testing the cell's surface tetrahedra j, j+LPP, ...: boxes overlap and
// no plane of the tetrahedron leaves the flux tet entirely outside.  The
// survivors (pair, surface tetrahedron, mask of cutting planes) are written in
// tetrahedron order into a range of the unit buffer reserved for the pair, so
// the result does not depend on LPP.
// Unit word: bits 0-15 the surface tetrahedron, 16-19 the mask of its
// planes that cut the flux tet, bit 16 + kUnitWideBit set when the first of
// those cuts keeps three tetrahedra.
__device__ inline unsigned unit_mask(unsigned code) { return (code >> 16) & 15u; }
// A pair's unit count carries this bit when its flux tet is negatively oriented (the sign of the pair's
// sum), so the per-pair sum needs no second look at the tet.
constexpr int kUcntNeg = 1 << 30;

template <int LPP>
__global__ __launch_bounds__(256) void k_flux_gen_filter(DevMesh M) {
  static_assert(LPP == 8 || LPP == 16 || LPP == 32 || LPP == 64, "lanes per pair");
  const int rsize = M.item_cap / kItemRegions, ursize = M.unit_cap / kItemRegions;
  const int r = blockIdx.x % kItemRegions, sub = blockIdx.x / kItemRegions;
  const int fill = region_items(M, r, rsize);
  const int hl = threadIdx.x & (LPP - 1), half = threadIdx.x / LPP;
  const int halves = blockDim.x / LPP;
  const int glead = threadIdx.x & 63 & ~(LPP - 1);  // first lane of the group within the wavefront
  const unsigned long long hmask = (LPP == 64 ? ~0ull : ((1ull << LPP) - 1ull)) << glead;
  for (int li = sub * halves + half; li < fill; li += region_blocks() * halves) {
    const int i = r * rsize + li;
    const int k = M.item_cell[i];
    if (M.isbox[k]) {
      if (hl == 0) M.item_ucnt[i] = -2;  // a box-cell pair has no units: the general-pair sum skips it
      continue;
    }
    unsigned tm = M.item_tm[i];
    Tet T = staged_tet(M, M.item_slot[i], tm);
    const d3 cc = cell_centre(M, k);
    d3 tlo = vmin(vmin(T.p0, T.p1), vmin(T.p2, T.p3)), thi = vmax(vmax(T.p0, T.p1), vmax(T.p2, T.p3));
    const int np = cell_piece_count(M, k);
    const bool tri_only = np == cf_count(M, k);
    const TetCont Tc = tet_container(T.p0, T.p1, T.p2, T.p3);
    const double sT = tet6(T);
    const bool live = sT != 0.0;  // a flat flux tet has no units
    double sc[4];
    apex_dists(Tc, cc, sc);
    // test of surface tetrahedron p against T: keep, and the mask of its planes that cut T
    auto test = [&](int p, unsigned& cm) -> bool {
      cm = 0;
      if (!live || p >= np) return false;
      d3 t0, t1, t2;
      cell_sigma(M, k, p, tri_only, t0, t1, t2);
      return unit_rule(T, tlo, thi, Tc, sc, cc, t0, t1, t2, cm);
    };
    // reserves count units (lane 0 of the group); -1 when the region is full
    auto reserve = [&](int count) -> int {
      int b = 0;
      if (hl == 0) {
        b = atomicAdd(&M.regions[r].unit_fill, count);
        if (b + count > ursize) {
          atomicMin(&M.regions[r].unit_okend, b);
          b = -1;
        } else {
          b += r * ursize;
        }
      }
      const int base = __shfl(b, glead, 64);
      if (hl == 0) {
        if (base < 0) {  // no room: the deferred kernel computes the whole pair
          M.item_ucnt[i] = -1;
          M.list_deep[atomicAdd(&M.counters[CNT_DEEP], 1)] = i;
        } else {
          M.item_uoff[i] = base;
          M.item_ucnt[i] = count | (sT < 0.0 ? kUcntNeg : 0);
        }
      }
      return base;
    };
    auto write_unit = [&](int u, int p, unsigned cm) {
      M.unit_item[u] = i;
      M.unit_code[u] = (unsigned)p | (cm << 16);
    };
    const unsigned long long below_mask = (1ull << __lane_id()) - 1ull;
    if (np <= 4 * LPP) {
      // up to four rounds: the tests stay in registers between counting and writing
      bool kq[4];
      unsigned cq[4];
      unsigned long long bq[4];
      int count = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        kq[q] = test(q * LPP + hl, cq[q]);
        bq[q] = __ballot(kq[q]) & hmask;
        count += __popcll(bq[q]);
      }
      const int base = reserve(count);
      if (base >= 0) {
        int written = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (kq[q]) write_unit(base + written + __popcll(bq[q] & below_mask), q * LPP + hl, cq[q]);
          written += __popcll(bq[q]);
        }
      }
    } else {
      // pass 0 counts, pass 1 writes into the reserved range
      int count = 0;
      for (int p0 = 0; p0 < np; p0 += LPP) {
        unsigned cm;
        count += __popcll(__ballot(test(p0 + hl, cm)) & hmask);
      }
      const int base = reserve(count);
      if (base >= 0) {
        int written = 0;
        for (int p0 = 0; p0 < np; p0 += LPP) {
          unsigned cm;
          const bool keep = test(p0 + hl, cm);
          const unsigned long long bm = __ballot(keep) & hmask;
          if (keep) write_unit(base + written + __popcll(bm & below_mask), p0 + hl, cm);
          written += __popcll(bm);
        }
      }
    }
  }
}

// Pairs with a general cell, stage 1 by runs (the default; k_flux_gen_filter
// gives the same units).  The staging kernel writes a face's pairs candidate
// by candidate, so the pairs of one face with one cell are consecutive in the
// pair buffer: a run, whose flux tets all meet the same surface tetrahedra.
// A block first scans its pairs, one per lane, for where runs start and end,
// and loads each run's cell data (piece count, vertex mean, the offset of its
// cached surface triangles) for all its runs at once.  A group of kRunLanes
// lanes then takes a run and
//  - stages up to kRunTets of its flux tets in LDS (vertices, box, inward
//    face planes, distances of the cell's vertex mean from those planes);
//  - gives each surface tetrahedron a lane, which loads it once for the run
//    and tests its box against every flux tet's;
//  - lists the (flux tet, surface tetrahedron) pairs whose boxes meet, flux
//    tet by flux tet in surface order, with the surface tetrahedron's
//    orientation, and gives the list's entries one lane each for the plane
//    tests of unit_rule (the rule every path applies);
//  - writes each pair's survivors in surface order into a range of the unit
//    buffer, taken from a pool the block reserves once per pass.
// So each pair gets the units k_flux_gen_filter gives it, in the same order.
// Cells with more than kRunLanes surface pieces leave their pairs to the
// deferred kernel.
// A block is one wavefront (two groups): its barriers then wait for no other
// wavefront, so a group's long run holds up only its partner.  Each block
// takes few pairs per pass and the grid has many blocks per region, so that
// the runs are spread over every CU rather than queued behind each other.
constexpr int kRunLanes = 32;
constexpr int kRunTets = 10;
constexpr int kRunBlock = 64;
constexpr int kRunGroups = kRunBlock / kRunLanes;
constexpr int kRunChunk = 64;             // pairs scanned for runs per block pass
constexpr int kRunPool = 90;              // units reserved per block pass, shared by the block's runs
constexpr int kRunBlocksPerRegion = 256;  // the grid: kItemRegions x this
struct RunLds {
  double tv[kRunTets][12];  // flux tet vertices
  double tp[kRunTets][16];  // inward face planes: normals n0..n3, then offsets d0..d3
  double tb[kRunTets][6];   // box: lo, hi
  unsigned short list[kRunTets * kRunLanes];  // flux tet << 8 | 32 if negatively oriented | surface tetrahedron
  unsigned char code[kRunTets * kRunLanes];   // survivor's unit word (cut mask, first-cut width, direction)
  double tsc[kRunTets][4];  // distances of the cell's vertex mean from each flux tet's face planes
  int seg[kRunTets + 1];                      // start of each flux tet's part of the list
  // survivors of the list's entries 32 j .. 32 j + 31 (bit per entry), and how many survive before them;
  // one word past the list's end holds no survivor
  unsigned keep[kRunTets + 1];
  int before[kRunTets + 1];
};
// Survivors among the first x entries of a run's list.
__device__ inline int run_survivors_before(const RunLds& S, int x) {
  const int j = x / kRunLanes, b = x % kRunLanes;
  return S.before[j] + __popc(S.keep[j] & ((1u << b) - 1u));
}
__device__ inline Tet run_tet(const RunLds& S, int t) {
  const double* v = S.tv[t];
  return Tet{mk3(v[0], v[1], v[2]), mk3(v[3], v[4], v[5]), mk3(v[6], v[7], v[8]), mk3(v[9], v[10], v[11])};
}
// Face plane l of the tetrahedron (a, b, c, d), as tet_container computes it
// (c and d already swapped for a negative orientation).
__device__ __forceinline__ Plane tet_face_plane(int l, d3 a, d3 b, d3 c, d3 d) {
  const d3 N = l == 0 ? crossf(c - a, b - a) : (l == 1 ? crossf(b - a, d - a) : (l == 2 ? crossf(d - a, c - a) : crossf(c - b, d - b)));
  return Plane{mk3(-N.x, -N.y, -N.z), dotf(N, l == 3 ? b : a)};
}
// unit_rule for entry (flux tet t, surface tetrahedron q0 q1 q2 about cc) of a
// run's list, which holds only pairs whose boxes meet and whose surface
// tetrahedron is not flat (neg: its orientation is negative).  The flux tet's
// data come from LDS as each test needs them; the surface tetrahedron's planes
// are computed one at a time by the fixed formulas tet_container applies
// (unrolled, so no plane is picked at run time).  The same operations on the
// same values as unit_rule, so the same decisions and the same unit word.
// (unit_rule's "largest distance <= 0" and "smallest distance < 0" as
// comparisons of the four distances: the same decisions for finite values,
// in compares that need no canonicalising of max / min operands)
__device__ __forceinline__ bool all_nonpos(double s0, double s1, double s2, double s3) {
  return s0 <= 0.0 && s1 <= 0.0 && s2 <= 0.0 && s3 <= 0.0;
}
__device__ __forceinline__ bool any_neg(double s0, double s1, double s2, double s3) {
  return s0 < 0.0 || s1 < 0.0 || s2 < 0.0 || s3 < 0.0;
}
__device__ __forceinline__ void run_forward_plane(const Plane& P, const Tet& T, int l, unsigned& cm, unsigned& wa,
                                                  bool& out) {
  const double s0 = P.dist(T.p0), s1 = P.dist(T.p1), s2 = P.dist(T.p2), s3 = P.dist(T.p3);
  if (all_nonpos(s0, s1, s2, s3)) out = true;
  if (any_neg(s0, s1, s2, s3)) {
    if (cm == 0u) wa = wide_bit(s0, s1, s2, s3);
    cm |= 1u << l;
  }
}
__device__ inline bool run_unit_rule(const RunLds& S, int t, bool neg, d3 cc, d3 q0, d3 q1, d3 q2, unsigned& word) {
  word = 0;
  unsigned cm = 0, wa = 0;
  {
    const Tet T = run_tet(S, t);
    const d3 a = cc, b = q0, c = neg ? q2 : q1, d = neg ? q1 : q2;
    bool out = false;
    run_forward_plane(tet_face_plane(0, a, b, c, d), T, 0, cm, wa, out);
    if (out) return false;
    run_forward_plane(tet_face_plane(1, a, b, c, d), T, 1, cm, wa, out);
    if (out) return false;
    run_forward_plane(tet_face_plane(2, a, b, c, d), T, 2, cm, wa, out);
    if (out) return false;
    run_forward_plane(tet_face_plane(3, a, b, c, d), T, 3, cm, wa, out);
    if (out) return false;
  }
  unsigned rm = 0, wb = 0;
  const double* q = S.tp[t];
#pragma unroll 1
  for (int l = 0; l < 4; ++l) {
    const Plane P{mk3(q[3 * l], q[3 * l + 1], q[3 * l + 2]), q[12 + l]};
    const double s0 = S.tsc[t][l], s1 = P.dist(q0), s2 = P.dist(q1), s3 = P.dist(q2);
    if (all_nonpos(s0, s1, s2, s3)) return false;
    if (any_neg(s0, s1, s2, s3)) {
      if (rm == 0u) wb = wide_bit(s0, s1, s2, s3);
      rm |= 1u << l;
    }
  }
  const bool flip = __popc(rm) < __popc(cm);
  word = flip ? (rm | (rm ? wb << kUnitWideBit : 0u) | (1u << kUnitFlipBit)) : (cm | (cm ? wa << kUnitWideBit : 0u));
  return true;
}

__global__ __launch_bounds__(kRunBlock, 3) void k_flux_gen_runs(DevMesh M) {
  static_assert(kRunChunk == kRunBlock && kRunBlock == 64, "the pass scans one pair per lane of its wavefront");
  __shared__ RunLds SS[kRunGroups];
  // the pass's runs, in pair order: first pair, length (0 when the run goes on past the pass's pairs), cell,
  // polyhedron slot, surface piece count, offset of the cell's cached surface triangles (-1: none), vertex mean
  __shared__ int s_head[kRunChunk], s_len[kRunChunk], s_cell[kRunChunk], s_slot[kRunChunk], s_np[kRunChunk];
  __shared__ int s_tro[kRunChunk];
  __shared__ double s_cc[kRunChunk][3];
  __shared__ unsigned short s_tm[kRunChunk];  // the pass's pairs' tetrahedron words
  // the block's pool of units: [s_pool, s_pool + kRunPool) of the unit buffer,
  // handed out to runs with LDS atomics (one device atomic per pass instead of
  // one per run); runs that do not fit take ranges of their own
  __shared__ int s_pool, s_pool_used, s_pool_fail;
  const int rsize = M.item_cap / kItemRegions, ursize = M.unit_cap / kItemRegions;
  const int r = blockIdx.x % kItemRegions, bsub = blockIdx.x / kItemRegions;
  const int fill = region_items(M, r, rsize);
  const int base = r * rsize;
  const int lane = __lane_id();
  const int grp = threadIdx.x / kRunLanes, sub = threadIdx.x & (kRunLanes - 1);
  const int gbase = lane & ~(kRunLanes - 1);  // the group's first lane in the wavefront
  const unsigned long long gmask = 0xffffffffull << gbase;
  const unsigned long long lbelow = ((1ull << lane) - 1ull) & gmask;
  RunLds& S = SS[grp];
  // every thread of a block makes the same number of passes (block barriers)
  for (int b = bsub * kRunChunk; b < fill; b += region_blocks() * kRunChunk) {
    // pairs b .. b + 63, one per lane: where runs start (a pair of another face or cell than the pair
    // before; past the filled pairs every lane counts as a start) and, for the first pair of each general
    // run, what the run needs of its cell, loaded at once for all the pass's runs
    int nh;
    {
      const int li = b + lane;
      bool brk = true, head = false;
      int k = 0, sl = 0;
      unsigned tm = 0;
      if (li < fill) {
        const int i = base + li;
        k = M.item_cell[i];
        sl = M.item_slot[i];
        tm = M.item_tm[i];
        brk = li == 0 || M.item_cell[i - 1] != k || M.item_slot[i - 1] != sl;
        const bool box = M.any_box && M.isbox[k] != 0;
        if (box) M.item_ucnt[i] = -2;  // a box-cell pair has no units: the general-pair sum skips it
        head = brk && !box;
      }
      const unsigned long long bb = __ballot(brk), bh = __ballot(head);
      nh = __popcll(bh);
      if (head) {
        const int h = __popcll(bh & ((1ull << lane) - 1ull));
        const unsigned long long after = lane < 63 ? bb >> (lane + 1) : 0ull;
        const int np = cell_piece_count(M, k);
        const int o = M.tri_off[k], o1 = M.tri_off[k + 1];
        s_head[h] = li;
        s_len[h] = after ? 1 + __builtin_ctzll(after) : 0;
        s_cell[h] = k;
        s_slot[h] = sl;
        s_np[h] = np;
        s_tro[h] = (o1 > o && np == cf_count(M, k)) ? o : -1;
        s_cc[h][0] = M.ccx[k];
        s_cc[h][1] = M.ccy[k];
        s_cc[h][2] = M.ccz[k];
      }
      s_tm[lane] = (unsigned short)tm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_pool = -1;
      s_pool_used = 0;
      s_pool_fail = 0;
      if (nh > 0) {
        const int pb = atomicAdd(&M.regions[r].unit_fill, kRunPool);
        if (pb + kRunPool > ursize) {
          atomicMin(&M.regions[r].unit_okend, pb);  // the region's written part ends before the pool
        } else {
          s_pool = r * ursize + pb;
          s_pool_fail = kRunPool;
        }
      }
    }
    __syncthreads();
    for (int hh = grp; hh < nh; hh += kRunGroups) {  // group-uniform from here on
      const int li0 = s_head[hh];
      const int i0 = base + li0;
      const int k = s_cell[hh], sl = s_slot[hh], np = s_np[hh], tro = s_tro[hh];
      // run length: the following pairs of the same face and cell (at most 5 kMaxFaceVerts), known from the
      // pass's starts unless the run goes on past the pass's pairs
      int R = s_len[hh];
      if (R == 0) {
        R = 1;
        for (int j0 = 1;; j0 += kRunLanes) {
          const int lj = li0 + j0 + sub;
          const bool same = lj < fill && M.item_cell[base + lj] == k && M.item_slot[base + lj] == sl;
          const unsigned long long bm = (__ballot(same) & gmask) >> gbase;
          const int lead = __builtin_ctzll(~bm);
          R += lead;
          if (lead < kRunLanes) break;
        }
      }
      if (np > kRunLanes) {  // more surface pieces than lanes: the deferred kernel takes these pairs
        for (int t = sub; t < R; t += kRunLanes) {
          M.item_ucnt[i0 + t] = -1;
          M.list_deep[atomicAdd(&M.counters[CNT_DEEP], 1)] = i0 + t;
        }
        continue;
      }
      const d3 cc = mk3(s_cc[hh][0], s_cc[hh][1], s_cc[hh][2]);
      // surface tetrahedron p: from the cell's cached triangles when it has them
      auto sigma = [&](int p, d3& t0, d3& t1, d3& t2) {
        if (tro >= 0) {
          const double* q = M.tri_xyz + 9 * (size_t)(tro + p);
          t0 = mk3(q[0], q[1], q[2]);
          t1 = mk3(q[3], q[4], q[5]);
          t2 = mk3(q[6], q[7], q[8]);
        } else {
          cell_sigma(M, k, p, np == cf_count(M, k), t0, t1, t2);
        }
      };
      for (int c0 = 0; c0 < R; c0 += kRunTets) {
        const int Rc = min(kRunTets, R - c0);
        // the run's flux tets, staged in steps so that few values are live at once
        bool dead = true, negt = false;
        if (sub < Rc) {
          const int lt = li0 - b + c0 + sub;
          const Tet T = staged_tet(M, sl, lt < kRunChunk ? (unsigned)s_tm[lt] : (unsigned)M.item_tm[i0 + c0 + sub]);
          const d3 tlo = vmin(vmin(T.p0, T.p1), vmin(T.p2, T.p3)), thi = vmax(vmax(T.p0, T.p1), vmax(T.p2, T.p3));
          double* v = S.tv[sub];
          v[0] = T.p0.x; v[1] = T.p0.y; v[2] = T.p0.z; v[3] = T.p1.x; v[4] = T.p1.y; v[5] = T.p1.z;
          v[6] = T.p2.x; v[7] = T.p2.y; v[8] = T.p2.z; v[9] = T.p3.x; v[10] = T.p3.y; v[11] = T.p3.z;
          double* bx = S.tb[sub];
          bx[0] = tlo.x; bx[1] = tlo.y; bx[2] = tlo.z; bx[3] = thi.x; bx[4] = thi.y; bx[5] = thi.z;
          const double sT = tet6(T);
          dead = sT == 0.0;
          negt = sT < 0.0;
        }
        wave_lds_sync();
        if (sub < Rc) {  // face planes, as tet_container computes them, one at a time
          const Tet T = run_tet(S, sub);
          const bool swp = det3f(T.p1 - T.p0, T.p2 - T.p0, T.p3 - T.p0) < 0.0;
          const d3 a = T.p0, b = T.p1, c = swp ? T.p3 : T.p2, d = swp ? T.p2 : T.p3;
          double* q = S.tp[sub];
#pragma unroll
          for (int l = 0; l < 4; ++l) {  // (each plane by its fixed formula, stored before the next)
            const Plane P = tet_face_plane(l, a, b, c, d);
            q[3 * l] = P.n.x; q[3 * l + 1] = P.n.y; q[3 * l + 2] = P.n.z; q[12 + l] = P.d;
            S.tsc[sub][l] = P.dist(cc);
          }
        }
        wave_lds_sync();  // flux tets staged (the group is within one wavefront)
        const unsigned deadm = (unsigned)((__ballot(dead) & gmask) >> gbase);
        // boxes: bit t set when flux tet t's box meets this lane's surface tetrahedron's
        unsigned pb = 0;
        d3 t0 = cc, t1 = cc, t2 = cc;
        bool flat = true, neg = false;
        if (sub < np) {
          sigma(sub, t0, t1, t2);
          const double s6 = det3f(t0 - cc, t1 - cc, t2 - cc);
          flat = s6 == 0.0;
          neg = s6 < 0.0;
        }
        const d3 slo = vmin(vmin(cc, t0), vmin(t1, t2)), shi = vmax(vmax(cc, t0), vmax(t1, t2));
        if (sub < np && !flat) {
          for (int t = 0; t < Rc; ++t) {
            if ((deadm >> t) & 1u) continue;
            const double* bx = S.tb[t];
            if (box_overlap(mk3(bx[0], bx[1], bx[2]), mk3(bx[3], bx[4], bx[5]), slo, shi)) pb |= 1u << t;
          }
        }
        // the list, flux tet by flux tet, each in surface order
        int ncombo = 0;
        for (int t = 0; t < Rc; ++t) {
          const bool in = (pb >> t) & 1u;
          const unsigned long long bt = __ballot(in) & gmask;
          if (sub == 0) S.seg[t] = ncombo;
          if (in) S.list[ncombo + __popcll(bt & lbelow)] = (unsigned short)((t << 8) | (neg ? 32u : 0u) | sub);
          ncombo += __popcll(bt);
        }
        if (sub == 0) S.seg[Rc] = ncombo;
        wave_lds_sync();
        // plane tests, one entry per lane, 32 entries a round; each round's survivors as a bit word, and
        // the count of survivors before it
        const int nw = (ncombo + kRunLanes - 1) / kRunLanes;
        int total = 0;
        for (int j = 0; j < nw; ++j) {
          const int c = j * kRunLanes + sub;
          bool keep = false;
          if (c < ncombo) {
            const unsigned e = S.list[c];
            const int t = (int)(e >> 8), p = (int)(e & 31u);
            d3 q0, q1, q2;
            sigma(p, q0, q1, q2);
            unsigned cm;
            keep = run_unit_rule(S, t, (e & 32u) != 0u, cc, q0, q1, q2, cm);
            S.code[c] = (unsigned char)cm;
          }
          const unsigned kw = (unsigned)((__ballot(keep) & gmask) >> gbase);
          if (sub == 0) {
            S.keep[j] = kw;
            S.before[j] = total;
          }
          total += __popc(kw);
        }
        if (sub == 0) {
          S.keep[nw] = 0u;
          S.before[nw] = total;
        }
        wave_lds_sync();
        // the run's units are its survivors in list order (flux tet by flux tet, each in surface order), so a
        // survivor's unit is the run's first plus the survivors before it, and a pair's units start at the
        // survivors before its part of the list
        int first = 0, cnt = 0;
        if (sub < Rc) {
          first = run_survivors_before(S, S.seg[sub]);
          cnt = run_survivors_before(S, S.seg[sub + 1]) - first;
        }
        int ub = 0;
        if (sub == 0 && total > 0) {
          const int o = s_pool >= 0 ? atomicAdd(&s_pool_used, total) : kRunPool;
          if (o + total <= kRunPool) {
            ub = s_pool + o;
          } else {
            if (s_pool >= 0) atomicMin(&s_pool_fail, o);  // the pool's used part ends before this request
            ub = atomicAdd(&M.regions[r].unit_fill, total);
            if (ub + total > ursize) {
              atomicMin(&M.regions[r].unit_okend, ub);  // the region's written part ends before this range
              ub = -1;
            } else {
              ub += r * ursize;
            }
          }
        }
        ub = __shfl(ub, 0, kRunLanes);
        if (sub < Rc) {
          const int i = i0 + c0 + sub;
          if (ub < 0) {  // no room: the deferred kernel computes the whole pair
            M.item_ucnt[i] = -1;
            M.list_deep[atomicAdd(&M.counters[CNT_DEEP], 1)] = i;
          } else {
            M.item_uoff[i] = ub + first;
            M.item_ucnt[i] = cnt | (negt ? kUcntNeg : 0);
          }
        }
        wave_lds_sync();
        if (ub >= 0) {
          for (int j = 0; j < nw; ++j) {
            const unsigned kw = S.keep[j];
            if ((kw >> sub) & 1u) {
              const int c = j * kRunLanes + sub;
              const unsigned e = S.list[c];
              const int u = ub + S.before[j] + __popc(kw & ((1u << sub) - 1u));
              M.unit_item[u] = i0 + c0 + (int)(e >> 8);
              M.unit_code[u] = (e & 31u) | ((unsigned)S.code[c] << 16);
            }
          }
        }
        wave_lds_sync();  // the group's LDS is reused by its next chunk or run
      }
    }
    __syncthreads();
    if (s_pool >= 0) {  // the pool's unused tail: units that no pair owns
      const int end = min(s_pool_used, s_pool_fail);
      for (int u = end + threadIdx.x; u < kRunPool; u += kRunBlock) M.unit_item[s_pool + u] = -1;
    }
    __syncthreads();  // s_head and the pool are reused by the next pass
  }
}

// Stage 2: one lane per surviving (pair, surface tetrahedron): clip in
// registers, up to three cutting planes; units with four (about 5% on the
// distorted-grid workload) go to a list for k_flux_gen_units_deep, which runs
// the same register clip one level deeper (so every unit has one value
// whichever kernel computes it).
// kUnitsPerThread units per thread are ranked together (a launch shape: 4 or 8,
// kItemsBlock x this units a block pass; a wider window gives more wavefronts
// of one kind where the units are mixed, as in a batch of many problems, at
// the cost of longer passes).
template <int kUnitsPerThread>
__global__ __launch_bounds__(kItemsBlock) void k_flux_gen_units(DevMesh M) {
  // As in the box-pair kernel, each block ranks its units by their work (the
  // number of cutting planes, 0..3, and whether the cell's interface cuts the
  // leaves) before clipping, so that most wavefronts run one kind of unit.
  // The ranking pass also loads what the clip needs of each unit's pair
  // (cell, polyhedron slot, tetrahedron word, the cell's cached surface
  // triangles), for its kUnitsPerThread units at once, and keeps it with the
  // rank in LDS: the clip then waits for one round of loads instead of three
  // in a row.
  constexpr int NCLS = 14;  // none; then per cut count 1..3, first cut keeping one or three; x interface
  constexpr int CHUNK = kItemsBlock * kUnitsPerThread;
  constexpr int VW = CHUNK / 64;
  // per unit, at its place in the pass (h kItemsBlock + thread): what the clip needs; s_list, in rank order,
  // holds those places
  __shared__ int s_unit[CHUNK], s_cell[CHUNK], s_slot[CHUNK], s_tri[CHUNK], s_list[CHUNK];
  __shared__ unsigned s_code[CHUNK];
  __shared__ unsigned short s_tm[CHUNK];
  __shared__ int s_off[VW][NCLS];
  __shared__ int s_n;
  const int rsize = M.unit_cap / kItemRegions;
  const int r = blockIdx.x % kItemRegions, sub = blockIdx.x / kItemRegions;
  const int fill = min(min(M.regions[r].unit_fill, M.regions[r].unit_okend), rsize);
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  // every thread of a block makes the same number of passes (block barriers)
  for (int b = sub * CHUNK; b < fill; b += region_blocks() * CHUNK) {
    int cls[kUnitsPerThread];
    unsigned long long mh[kUnitsPerThread];
#pragma unroll
    for (int h = 0; h < kUnitsPerThread; ++h) {
      const int lu = b + threadIdx.x + h * kItemsBlock;
      const int u = r * rsize + lu;
      int c = -1, i = -1, k = 0, sl = 0, tro = -1;
      unsigned code = 0, tm = 0;
      if (lu < fill) {
        i = M.unit_item[u];
        code = M.unit_code[u];
      }
      if (i >= 0) {  // (units of no pair, the unused tail of a block's pool, are skipped)
        k = M.item_cell[i];
        sl = M.item_slot[i];
        tm = M.item_tm[i];
        const int nc = cut_count(unit_mask(code));
        const int8_t tg = M.tag_cell[k];
        // the surface triangle's place in the bind-time cache, when the cell's pieces are its triangles
        // and they are cached (else -1: the clip builds the piece itself)
        const int o = M.tri_off[k], o1 = M.tri_off[k + 1];
        tro = (o1 > o && cf_count(M, k) == cell_piece_count(M, k)) ? o + (int)(code & 0xffffu) : -1;
        const int wide = (int)((code >> (16 + kUnitWideBit)) & 1u);
        if (nc > 3) M.list_udeep[atomicAdd(&M.counters[CNT_UDEEP], 1)] = u;  // four cutting planes: the deep instance
        else c = nc == 0 ? (tg == 0 ? 1 : 0) : 2 + 4 * (nc - 1) + 2 * wide + (tg == 0 ? 1 : 0);
      }
      unsigned long long m = 0;
#pragma unroll
      for (int q = 0; q < NCLS; ++q) {
        const unsigned long long bq = __ballot(c == q);
        if (lane == 0) s_off[h * (kItemsBlock / 64) + w][q] = __popcll(bq);
        m = c == q ? bq : m;
      }
      cls[h] = c;
      mh[h] = m;
      const int raw = h * kItemsBlock + threadIdx.x;
      s_unit[raw] = u;
      s_cell[raw] = k;
      s_slot[raw] = sl;
      s_tri[raw] = tro;
      s_code[raw] = code;
      s_tm[raw] = (unsigned short)tm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int c = NCLS - 1; c >= 0; --c)
        for (int v = 0; v < VW; ++v) {
          const int n = s_off[v][c];
          s_off[v][c] = t;
          t += n;
        }
      s_n = t;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < kUnitsPerThread; ++h) {
      if (cls[h] >= 0) s_list[s_off[h * (kItemsBlock / 64) + w][cls[h]] + __popcll(mh[h] & below)] = h * kItemsBlock + threadIdx.x;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < s_n; q += kItemsBlock) {  // ranks in order of work, most first
      const int raw = s_list[q];
      const int uu = s_unit[raw], k = s_cell[raw], tro = s_tri[raw];
      const unsigned cd = s_code[raw];
      const int p = cd & 0xffff;
      const unsigned w = (cd >> 16) & 63u;
      const Tet T = staged_tet(M, s_slot[raw], s_tm[raw]);
      const d3 cc = cell_centre(M, k);
      d3 t0, t1, t2;
      if (tro >= 0) {
        const double* tq = M.tri_xyz + 9 * (size_t)tro;
        t0 = mk3(tq[0], tq[1], tq[2]);
        t1 = mk3(tq[3], tq[4], tq[5]);
        t2 = mk3(tq[6], tq[7], tq[8]);
      } else {
        cell_sigma(M, k, p, cf_count(M, k) == cell_piece_count(M, k), t0, t1, t2);
      }
      const double s6 = det3f(t0 - cc, t1 - cc, t2 - cc);
      Tet X;
      TetCont C;
      unit_clip_value_setup(T, cc, t0, t1, t2, w, X, C);
      Leaf leaf;
      leaf.useH = M.tag_cell[k] == 0;
      leaf.hn = mk3(M.pnx[k], M.pny[k], M.pnz[k]);
      leaf.hd = M.pC[k];
      const double v = clip_masked_tet<3, false>(X, C, w & 15u, leaf);
      M.unit_vol[uu] = s6 > 0.0 ? v : -v;
    }
    __syncthreads();  // the lists are reused by the next pass
  }
}

__global__ __launch_bounds__(256) void k_flux_gen_units_deep(DevMesh M) {
  const int n = M.counters[CNT_UDEEP];
  for (int j = grid_stride_start(); j < n; j += grid_stride()) {
    const int u = M.list_udeep[j];
    const int i = M.unit_item[u];
    const unsigned code = M.unit_code[u];
    const int k = M.item_cell[i];
    Tet T = staged_tet(M, M.item_slot[i], M.item_tm[i]);
    const d3 cc = cell_centre(M, k);
    const bool tri_only = cf_count(M, k) == cell_piece_count(M, k);
    d3 t0, t1, t2;
    cell_sigma(M, k, code & 0xffff, tri_only, t0, t1, t2);
    double s6 = det3f(t0 - cc, t1 - cc, t2 - cc);
    const unsigned w = (code >> 16) & 63u;
    Tet X;
    TetCont C;
    unit_clip_value_setup(T, cc, t0, t1, t2, w, X, C);
    Leaf leaf;
    leaf.useH = M.tag_cell[k] == 0;
    leaf.hn = mk3(M.pnx[k], M.pny[k], M.pnz[k]);
    leaf.hd = M.pC[k];
    // all four planes cut (the unit kernel takes the others): the first split's children in a loop, each
    // clipped by the expanded three-plane form, with the values and the order of the sums of the looping
    // form every other path uses (clip_masked_tet<4>).  Looping every level was a quarter slower, the
    // expanded form at every level slower still; the planes are taken from the container inside the
    // loop, which kept them out of the registers live across it (160 against 187 us on 64^3 distorted).
    double v = 0.0;
    {
      const Split sp = split_by(X, C.plane(0));
      const int n = sp.count();
      for (int i = 0; i < n; ++i) v += clip3(sp.child(i), C.plane(1), C.plane(2), C.plane(3), leaf);
    }
    M.unit_vol[u] = s6 > 0.0 ? v : -v;
  }
}

// Stage 3: per pair, the sum of its units in surface-tetrahedron order, signed by the flux tet.
__global__ __launch_bounds__(256) void k_flux_gen_sum(DevMesh M) {
  const int rsize = M.item_cap / kItemRegions;
  const int r = blockIdx.x % kItemRegions, sub = blockIdx.x / kItemRegions;
  const int fill = region_items(M, r, rsize);
  for (int li = sub * blockDim.x + threadIdx.x; li < fill; li += region_blocks() * blockDim.x) {
    const int i = r * rsize + li;
    const int cw = M.item_ucnt[i];
    if (cw < 0) continue;  // a box-cell pair (-2) or a deferred one (-1)
    const int cnt = cw & (kUcntNeg - 1);
    // the units eight at a time, loads in flight together and added in order
    const double* v = M.unit_vol + M.item_uoff[i];
    double acc = 0.0;
    int q = 0;
    for (; q + 8 <= cnt; q += 8) {
      double t[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) t[j] = v[q + j];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += t[j];
    }
    for (; q < cnt; ++q) acc += v[q];
    M.item_vol[i] = (cw & kUcntNeg) ? -acc : acc;
  }
}

// Signed volume of one (flux tet, box cell) pair with cut mask `mask`: the
// value every kernel gives the pair (the looping form of the register clip up
// to four cutting planes, equal bit for bit to the expanded form the pair
// kernel runs up to kMaxRegCuts; the explicit-stack clip beyond; a flat flux
// tet gives 0).
__device__ __attribute__((always_inline)) inline double box_pair_volume(const DevMesh& M, const Tet& T, const BoxCont& B, unsigned mask,
                                         const Leaf& leaf) {
  double sT = tet6(T);
  if (sT == 0.0) return 0.0;
  const int nc = cut_count(mask);
  double v = nc <= 4 ? clip_masked_compact(T, B, mask, leaf) : clip_volume(T, B, leaf);
  if (v == -1.0) {
    atomicOr(&M.counters[CNT_ERR], ERR_STACK);
    v = 0.0;
  }
  return sT < 0.0 ? -v : v;
}

// Signed volume of one (flux tet, general cell) pair: the cell's surface
// tetrahedra in order, each clipped in registers (the same units and the same
// order as the three-stage path).
__device__ __attribute__((always_inline)) inline double general_pair_volume(const DevMesh& M, int k, d3 cc, const Tet& T, const Leaf& leaf) {
  double sT = tet6(T);
  if (sT == 0.0) return 0.0;
  double v;
  tet_cell_pieces_volume<true>(M, k, cc, T, leaf, v);
  return sT < 0.0 ? -v : v;
}

// Box pair with three or four cutting planes, computed by a group of
// kDeepLanes lanes: lane 3i + j takes grandchild j of child i of the first
// two splits and clips it by the remaining planes; the group then adds the
// parts level by level in child order, each level's sum starting from zero,
// which is exactly the association of the serial looping clip (the overflow
// kernel's), so both paths give the same bits.
constexpr int kDeepLanes = 16;
__device__ inline double box_pair_volume_group(const Tet& T, const BoxCont& B, unsigned mask, int nc,
                                               const Leaf& leaf, int sub, int gbase) {
  const double sT = tet6(T);
  if (sT == 0.0) return 0.0;
  Plane P0 = {}, P1 = {}, P2 = {}, P3 = {};
  unsigned rest = mask;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (rest) {
      const int l = __builtin_ctz(rest);
      rest &= rest - 1u;
      const Plane pl = B.plane(l);
      P0 = q == 0 ? pl : P0;
      P1 = q == 1 ? pl : P1;
      P2 = q == 2 ? pl : P2;
      P3 = q == 3 ? pl : P3;
    }
  }
  const int ci = sub / 3, cj = sub - 3 * ci;
  const Split s1 = split_by(T, P0);
  const int n1 = s1.count();
  double d = 0.0;
  int n2 = 0;
  if (sub < 9 && ci < n1) {
    const Split s2 = split_by(s1.child(ci), P1);
    n2 = s2.count();
    if (cj < n2) {
      const Tet g = s2.child(cj);
      d = nc == 3 ? clip1(g, P2, leaf) : clip2c(g, P2, P3, leaf);
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int na = __shfl(n2, gbase + 3 * a);
    double ca = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double db = __shfl(d, gbase + 3 * a + b);
      if (b < na) ca += db;
    }
    if (a < n1) acc += ca;
  }
  return sT < 0.0 ? -acc : acc;
}

// General pair computed by a group of kDeepLanes lanes: lane sub takes the
// cell's surface pieces sub, sub + kDeepLanes, ...; each piece's signed volume
// is computed as in the serial sum over the pieces, and the group adds the
// kept pieces in piece order (the serial sum's order, so the same bits).
__device__ inline double general_pair_volume_group(const DevMesh& M, int k, d3 cc, const Tet& T, const Leaf& leaf,
                                                   int sub, int gbase) {
  const double sT = tet6(T);
  if (sT == 0.0) return 0.0;
  const d3 tlo = vmin(vmin(T.p0, T.p1), vmin(T.p2, T.p3)), thi = vmax(vmax(T.p0, T.p1), vmax(T.p2, T.p3));
  const int np = cell_piece_count(M, k);
  const bool tri_only = np == cf_count(M, k);
  double acc = 0.0;
  const TetCont Tc = tet_container(T.p0, T.p1, T.p2, T.p3);
  double sc[4];
  apex_dists(Tc, cc, sc);
  for (int p0 = 0; p0 < np; p0 += kDeepLanes) {
    const int p = p0 + sub;
    bool kept = false;
    double val = 0.0;
    if (p < np) {
      d3 t0, t1, t2;
      cell_sigma(M, k, p, tri_only, t0, t1, t2);
      unsigned w;
      if (unit_rule(T, tlo, thi, Tc, sc, cc, t0, t1, t2, w)) {
        const double s6 = det3f(t0 - cc, t1 - cc, t2 - cc);
        Tet X;
        TetCont C;
        unit_clip_value_setup(T, cc, t0, t1, t2, w, X, C);
        const double v = clip_masked_tet(X, C, w & 15u, leaf);
        val = s6 > 0.0 ? v : -v;
        kept = true;
      }
    }
    const int nq = min(kDeepLanes, np - p0);
    for (int q = 0; q < nq; ++q) {
      const double vq = __shfl(val, gbase + q);
      if (__shfl((int)kept, gbase + q)) acc += vq;
    }
  }
  return sT < 0.0 ? -acc : acc;
}

// Deferred pairs, a group of kDeepLanes lanes per pair: box pairs with more
// cutting planes than the register clip takes, and general pairs whose units
// did not fit the unit buffer.
__global__ __launch_bounds__(64) void k_flux_deep(DevMesh M) {
  const int n = M.counters[CNT_DEEP];
  const int sub = threadIdx.x & (kDeepLanes - 1);
  const int gbase = __lane_id() & ~(kDeepLanes - 1);
  const int ngroups = (gridDim.x * blockDim.x) / kDeepLanes;
  // the trip count is the same for every lane of a group (the shuffles need all of them)
  for (int j = (blockIdx.x * blockDim.x + threadIdx.x) / kDeepLanes; j < n; j += ngroups) {
    const int i = M.list_deep[j];
    const int k = M.item_cell[i];
    const unsigned tm = M.item_tm[i];
    const Tet T = staged_tet(M, M.item_slot[i], tm);
    Leaf leaf;
    leaf.useH = M.tag_cell[k] == 0;
    leaf.hn = mk3(M.pnx[k], M.pny[k], M.pnz[k]);
    leaf.hd = M.pC[k];
    double v = 0.0;
    if (M.isbox[k]) {
      const BoxCont B{mk3(M.lox[k], M.loy[k], M.loz[k]), mk3(M.hix[k], M.hiy[k], M.hiz[k])};
      const unsigned mask = tm_mask(tm);
      const int nc = cut_count(mask);
      if (nc == 3 || nc == 4) v = box_pair_volume_group(T, B, mask, nc, leaf, sub, gbase);
      else if (sub == 0) v = box_pair_volume(M, T, B, mask, leaf);
    } else {
      v = general_pair_volume_group(M, k, cell_centre(M, k), T, leaf, sub, gbase);
    }
    if (sub == 0) M.item_vol[i] = v;
  }
}

// Per staged face: V_F = sum of its pairs in their fixed order (grid-strided).
__device__ inline void staged_face_sums(const DevMesh& M) {
  int n = min(M.counters[CNT_FACES], M.poly_cap);
  for (int it = grid_stride_start(); it < n; it += grid_stride()) {
    const int cnt = M.item_cnt[it], off = M.item_off[it], f = M.list_faces[it];
    if (cnt < 0) continue;
    const double* v = M.item_vol + off;
    double acc = 0.0;
    int i = 0;
    for (; i + 8 <= cnt; i += 8) {  // eight loads in flight, added in order
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = v[i + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += t[q];
    }
    for (; i < cnt; ++i) acc += v[i];
    M.VF[f] = acc;
  }
}

// Faces that did not fit the staging buffers (or have more candidate cells
// than the staging LDS holds): one wavefront per face, one lane per
// (candidate, flux tet) pair computing the pair's volume with the same
// functions as the staged path, summed in the same (candidate, tetrahedron)
// order, so V_F does not depend on which path computed it.
__device__ inline void overflow_faces(const DevMesh& M, FluxLds& S, const double* __restrict__ vel, double dt) {
  const int lane = threadIdx.x;
  const int nfaces = M.counters[CNT_OVER];
  for (int it = blockIdx.x; it < nfaces; it += gridDim.x) {
    const int f = M.list_over[it];
    const int b0 = fv_begin(M, f), I = fv_count(M, f);
    d3 c, Sv, plo, phi;
    flux_polyhedron(M, S, f, b0, I, vel, face_dt(M, f, dt), c, Sv, plo, phi);
    {  // coverage, as in the staging kernel, over every listed cell
      const int npt = slot_points(M.method, I);
      const int o = M.owner[f], nbr = M.neigh[f];
      const int ob = M.nb_ptr[o], on = M.nb_ptr[o + 1] - ob;
      const int nbb = nbr >= 0 ? M.nb_ptr[nbr] : 0, nbn = nbr >= 0 ? M.nb_ptr[nbr + 1] - nbb : 0;
      const int L = 1 + on + (nbr >= 0 ? 1 + nbn : 0);
      unsigned cov = outside_bits(M, S, f, I, npt, c);
      for (int j = lane; j < L; j += kFluxLanes) {
        const int k = candidate_cell(M, j, o, ob, on, nbr, nbb);
        cov |= cover_bits(S, I, npt, c, mk3(M.lox[k], M.loy[k], M.loz[k]), mk3(M.hix[k], M.hiy[k], M.hiz[k]));
      }
      for (int o2 = 1; o2 < kFluxLanes; o2 <<= 1) cov |= __shfl_xor(cov, o2);
      if (lane == 0 && (cov & needed_bits(I, npt)) != needed_bits(I, npt)) atomicOr(&M.counters[CNT_ERR], ERR_COVER);
    }
    const int ncand = flux_candidates(M, S, f, plo, phi);
    const int TF = flux_tet_count(M.method, I);
    const int total = ncand * TF;
    double acc = 0.0;  // identical in every lane
    for (int q0 = 0; q0 < total; q0 += kFluxLanes) {
      const int q = q0 + lane;
      int keep = 0;
      double v = 0.0;
      if (q < total) {
        const int t = q % TF, kc = q / TF;
        int i1, i2, i3;
        flux_tet_points(t, I, M.method, i1, i2, i3);
        Tet T{c, mk3(S.px[i1], S.py[i1], S.pz[i1]), mk3(S.px[i2], S.py[i2], S.pz[i2]),
              mk3(S.px[i3], S.py[i3], S.pz[i3])};
        d3 tlo = vmin(vmin(T.p0, T.p1), vmin(T.p2, T.p3)), thi = vmax(vmax(T.p0, T.p1), vmax(T.p2, T.p3));
        BoxCont B{mk3(S.clox[kc], S.cloy[kc], S.cloz[kc]), mk3(S.chix[kc], S.chiy[kc], S.chiz[kc])};
        keep = box_overlap(tlo, thi, B.lo, B.hi) ? 1 : 0;
        Leaf leaf;
        leaf.useH = S.ctag[kc] == 0;
        leaf.hn = mk3(S.cpnx[kc], S.cpny[kc], S.cpnz[kc]);
        leaf.hd = S.cpc[kc];
        if (keep && S.cbox[kc]) {
          unsigned mask = 0;
          keep = cut_mask(T, B, mask) ? 1 : 0;
          if (keep) v = box_pair_volume(M, T, B, mask, leaf);
        } else if (keep) {
          v = general_pair_volume(M, S.cand[kc], mk3(S.cccx[kc], S.cccy[kc], S.cccz[kc]), T, leaf);
        }
      }
      const int nq = min(kFluxLanes, total - q0);
      for (int j = 0; j < nq; ++j) {
        double vj = __shfl(v, j);
        if (__shfl(keep, j)) acc += vj;
      }
    }
    if (lane == 0) M.VF[f] = acc;
    __syncthreads();
  }
}

// The end of the flux stage in one launch of kFluxLanes-thread blocks: V_F of
// the staged faces (grid-strided, a thread per face), then of the faces that
// went to the overflow path (a block per face).  Neither reads what the other
// writes.
// vel: the velocities the flux polyhedra are built from (vertex velocities,
// or face velocities for NMFPA).
__global__ __launch_bounds__(kFluxLanes) void k_flux_sum(DevMesh M, const double* __restrict__ vel, double dt) {
  __shared__ FluxLds S;
  if (blockIdx.x == 0 && threadIdx.x == 0) M.totals[1] += (unsigned long long)M.counters[CNT_FACES];
  staged_face_sums(M);
  overflow_faces(M, S, vel, dt);
}

__global__ void k_reset_advect(DevMesh M) { reset_advect_state(M); }

// ============================================================== LSGIR + plane constant
// A group of kReconLanes lanes per interfacial cell (one lane per cell leaves
// the GPU nearly idle: a few thousand cells, each a long dependent chain).
constexpr int kReconLanes = 16;

// Sum over the lanes of a group.  Each butterfly level adds a lane's value
// and its partner's, which gives the same bits on both lanes, so every lane
// of the group ends with the same sum, in a fixed order.
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = 1; o < kReconLanes; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// vol(cell ∩ {n.x >= s}) for a general cell: signed surface tetrahedra from
// the vertex mean, split over the group's lanes.
__device__ inline double general_level_volume(const DevMesh& M, int c, d3 n, d3 cen, double s, int sub, int np,
                                              bool tri_only) {
  const double lc = dotf(n, cen) - s;
  double acc = 0.0;
  for (int p = sub; p < np; p += kReconLanes) {
    d3 t0, t1, t2;
    cell_sigma(M, c, p, tri_only, t0, t1, t2);
    double v6 = det3f(t0 - cen, t1 - cen, t2 - cen);
    double fr = halfspace_fraction(lc, dotf(n, t0) - s, dotf(n, t1) - s, dotf(n, t2) - s);
    acc = fma(v6, fr, acc);
  }
  return group_sum(acc) * (1.0 / 6.0);
}

// Two instances: BOX handles the axis-aligned box cells, whose plane constant
// needs only the eight corner levels (held one per lane of the group, so the
// instance keeps no per-lane arrays), and !BOX the general cells.
// GIVEN: the LSFIR placement pass `pass`: cells whose fitted normal in
// lsfir_nn differs from the current one take it, with their plane constant;
// the others are left alone.  Otherwise the LSGIR pass.
template <bool BOX, bool GIVEN>
__global__ __launch_bounds__(128) void k_recon(DevMesh M, const double* __restrict__ F, int count_cells, int pass) {
  if (GIVEN && pass > 1 && M.lsfir_turned[pass - 1] == 0) return;
  const int ncell = M.counters[CNT_CELLS];
  if (count_cells && blockIdx.x == 0 && threadIdx.x == 0) M.totals[0] += (unsigned long long)ncell;
  const double beta = M.beta;
  const bool beta15 = beta == 1.5;
  const int sub = threadIdx.x & (kReconLanes - 1);
  const int gbase = __lane_id() & ~(kReconLanes - 1);  // first lane of the group in the wavefront
  const int ngroups = (gridDim.x * blockDim.x) / kReconLanes;
  // the trip count is the same for every lane of a group (the shuffles below need all of them)
  for (int it = (blockIdx.x * blockDim.x + threadIdx.x) / kReconLanes; it < ncell; it += ngroups) {
    const int c = M.list_cells[it];
    // every load that depends only on c, issued together; the empty asm takes
    // them all at once, which keeps the compiler from sinking each to its
    // first use (a round trip each)
    int isb = M.isbox[c];
    const d3 xc = cell_centre(M, c);
    double Fc = F[c];
    const int nb0 = M.nb_ptr[c], nnb = M.nb_ptr[c + 1] - nb0;
    double Vc = M.V[c];
    d3 blo = xc, bhi = xc;
    if constexpr (BOX) {
      blo = mk3(M.lox[c], M.loy[c], M.loz[c]);
      bhi = mk3(M.hix[c], M.hiy[c], M.hiz[c]);
    }
    asm volatile("" : "+v"(isb), "+v"(Fc), "+v"(Vc), "+v"(blo.x), "+v"(blo.y), "+v"(blo.z), "+v"(bhi.x),
                 "+v"(bhi.y), "+v"(bhi.z));
    if ((isb != 0) != BOX) continue;  // uniform over the group
    d3 n;
    if constexpr (GIVEN) {
      const int nc = M.nc;
      n = mk3(M.lsfir_nn[c], M.lsfir_nn[nc + c], M.lsfir_nn[2 * nc + c]);
      if (n.x == M.pnx[c] && n.y == M.pny[c] && n.z == M.pnz[c]) continue;  // unchanged (uniform over the group)
    } else {
    // ---- LSGIR: normal equations sum w^2 d d^T g = sum w^2 d dF, w = |d|^-beta.
    // The lanes gather the neighbours' terms, a round of kReconLanes at a time,
    // and every lane accumulates all terms in neighbour order: the sums keep the
    // order of a serial loop (which decides the normal where the gradient
    // vanishes to rounding, e.g. a lone filled cell).
    double a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0, r0 = 0, r1 = 0, r2 = 0;
    for (int r = 0; r < nnb; r += kReconLanes) {
      d3 d = mk3(0.0, 0.0, 0.0);
      double w2 = 0.0, df = 0.0;
      if (r + sub < nnb) {
        int k = M.nb_idx[nb0 + r + sub];
        d3 ck = cell_centre(M, k);
        double fk = F[k];
        asm volatile("" : "+v"(ck.x), "+v"(ck.y), "+v"(ck.z), "+v"(fk));  // both loads in flight together
        d = ck - xc;
        double d2 = dotf(d, d);
        w2 = beta15 ? 1.0 / (d2 * sqrt(d2)) : pow(d2, -beta);
        df = (fk - Fc) * w2;
      }
      const int nq = min(kReconLanes, nnb - r);
      for (int j = 0; j < nq; ++j) {
        const double dx = __shfl(d.x, gbase + j), dy = __shfl(d.y, gbase + j), dz = __shfl(d.z, gbase + j);
        const double wj = __shfl(w2, gbase + j), fj = __shfl(df, gbase + j);
        a00 = fma(wj * dx, dx, a00);
        a01 = fma(wj * dx, dy, a01);
        a02 = fma(wj * dx, dz, a02);
        a11 = fma(wj * dy, dy, a11);
        a12 = fma(wj * dy, dz, a12);
        a22 = fma(wj * dz, dz, a22);
        r0 = fma(fj, dx, r0);
        r1 = fma(fj, dy, r1);
        r2 = fma(fj, dz, r2);
      }
    }
    // adjugate solve (A symmetric positive definite): g ~ adj(A) r
    double c00 = fma(a11, a22, -a12 * a12), c01 = fma(a02, a12, -a01 * a22), c02 = fma(a01, a12, -a02 * a11);
    double c11 = fma(a00, a22, -a02 * a02), c12 = fma(a01, a02, -a00 * a12), c22 = fma(a00, a11, -a01 * a01);
    double det = fma(a00, c00, fma(a01, c01, a02 * c02));
    d3 g = mk3(fma(c00, r0, fma(c01, r1, c02 * r2)), fma(c01, r0, fma(c11, r1, c12 * r2)),
               fma(c02, r0, fma(c12, r1, c22 * r2)));
    if (det < 0.0) g = mk3(-g.x, -g.y, -g.z);
    double gg = dotf(g, g);
    n = (gg > 0.0 && det != 0.0) ? (1.0 / sqrt(gg)) * g : mk3(0.0, 0.0, 1.0);
    }
    // ---- plane constant: G(s) = vol(cell ∩ {n.x >= s}) = F V, G decreasing from V to 0
    // over the sorted vertex levels
    // the smaller of the fluid and empty volumes is matched: for F > 1/2 the
    // empty part {-n.x >= s} with (1 - F) V (1 - F exact there), the same
    // plane, evaluated with rounding relative to the small volume
    const bool flip = Fc > 0.5;
    const d3 ns = flip ? mk3(-n.x, -n.y, -n.z) : n;
    const double T = (flip ? 1.0 - Fc : Fc) * Vc;
    double s0, w, glo, ghi;
    if constexpr (BOX) {
      // lane sub holds the level of corner sub; every lane gathers all eight
      const d3 p = mk3((sub & 1) ? bhi.x : blo.x, (sub & 2) ? bhi.y : blo.y, (sub & 4) ? bhi.z : blo.z);
      const double bl = dotf(ns, p);
      double blev[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) blev[q] = __shfl(bl, gbase + q);
      // rank of this lane's level in ascending order (ties by corner index),
      // then the level of rank sub: the sorted levels, one per lane
      int rank = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) rank += (blev[q] < bl || (blev[q] == bl && q < sub)) ? 1 : 0;
      double lev = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (__shfl(rank, gbase + q) == sub) lev = blev[q];
      }
      // G at the eight levels, one per lane; the bracket is the last level with G >= T and the next
      const double gj = box_level_volume(blev, Vc, lev);
      int lo_i = 0;
      glo = __shfl(gj, gbase);
      for (int q = 1; q < 8; ++q) {
        double gq = __shfl(gj, gbase + q);
        if (gq >= T) {
          lo_i = q;
          glo = gq;
        }
      }
      const int hi_i = lo_i < 7 ? lo_i + 1 : 7;
      const double gh = __shfl(gj, gbase + hi_i);
      ghi = hi_i == 7 ? 0.0 : gh;
      s0 = __shfl(lev, gbase + lo_i);
      w = __shfl(lev, gbase + hi_i) - s0;
      if (w > 0.0) {
        // the two interior points of the bracket's cubic, on lanes 0 and 1
        const double sq = fma(w, (sub & 1) ? 2.0 / 3.0 : 1.0 / 3.0, s0);
        const double yq = box_level_volume(blev, Vc, sq);
        const double y1 = __shfl(yq, gbase), y2 = __shfl(yq, gbase + 1);
        s0 = cubic_root(s0, w, glo, y1, y2, ghi, T);
      }
    } else {
      double lev[kMaxLevels];
      int nl = 0;
      insert_sorted(lev, nl, dotf(ns, xc));
      for (int i = M.cv_ptr[c]; i < M.cv_ptr[c + 1] && nl < kMaxLevels; ++i)
        insert_sorted(lev, nl, dotf(ns, vert(M, M.cv_idx[i])));
      int fb = cf_begin(M, c), fn = cf_count(M, c);
      for (int i = 0; i < fn && nl < kMaxLevels; ++i) {
        int e = M.cf_idx[fb + i];
        int f = e >= 0 ? e : ~e;
        if (fv_count(M, f) > 3) insert_sorted(lev, nl, dotf(ns, mk3(M.fcx[f], M.fcy[f], M.fcz[f])));
      }
      if (sub == 0 && M.cv_ptr[c + 1] - M.cv_ptr[c] + 1 > kMaxLevels) atomicOr(&M.counters[CNT_ERR], ERR_LEVELS);
      const int np = cell_piece_count(M, c);
      const bool tri_only = np == fn;
      // bisection over the levels; every evaluation is spread over the group
      int lo_i = 0, hi_i = nl - 1;
      glo = general_level_volume(M, c, ns, xc, lev[0], sub, np, tri_only);
      ghi = 0.0;
      while (hi_i - lo_i > 1) {
        int mid = (lo_i + hi_i) >> 1;
        double gm = general_level_volume(M, c, ns, xc, lev[mid], sub, np, tri_only);
        if (gm >= T) {
          lo_i = mid;
          glo = gm;
        } else {
          hi_i = mid;
          ghi = gm;
        }
      }
      s0 = lev[lo_i];
      w = lev[hi_i] - s0;
      if (w > 0.0) {
        double y1 = general_level_volume(M, c, ns, xc, fma(w, 1.0 / 3.0, s0), sub, np, tri_only);
        double y2 = general_level_volume(M, c, ns, xc, fma(w, 2.0 / 3.0, s0), sub, np, tri_only);
        s0 = cubic_root(s0, w, glo, y1, y2, ghi, T);
      }
    }
    if (sub == 0) {
      M.pnx[c] = n.x;
      M.pny[c] = n.y;
      M.pnz[c] = n.z;
      M.pC[c] = flip ? s0 : -s0;  // fluid {n.x >= -s0}, or the complement of {-n.x >= s0}
    }
  }
}

// ============================================================== LSFIR
// (Sec. "Least squares fit interface reconstruction")

// PLIC centres of the interfacial cells' current planes, a group of
// kReconLanes lanes per cell: the vertex mean of the polygon {n.x + C = 0}
// within the cell, i.e. of the cell's vertices on the plane (a lane per
// vertex) and of the strict crossings of its edges (a lane per face, over
// the face's edges).  Each edge is taken once, from the face in which the
// cell's outward orientation runs it from the lower vertex index to the
// higher (on a closed, consistently oriented cell exactly one of its two
// faces does).  Signed distances in the exact-order form, crossing points
// without contraction, group sums in a fixed order.  No point: the cell
// centre.  Runs before the first LSFIR pass and after each placement pass
// in which some normal turned.
__global__ __launch_bounds__(128) void k_plic_centres(DevMesh M, int pass) {
  if (pass > 0 && M.lsfir_turned[pass] == 0) return;  // no plane moved
  const int ncell = M.counters[CNT_CELLS];
  const int nc = M.nc;
  const int sub = threadIdx.x & (kReconLanes - 1);
  const int ngroups = (gridDim.x * blockDim.x) / kReconLanes;
  for (int it = (blockIdx.x * blockDim.x + threadIdx.x) / kReconLanes; it < ncell; it += ngroups) {
    const int c = M.list_cells[it];
    const d3 n = mk3(M.pnx[c], M.pny[c], M.pnz[c]);
    const double C = M.pC[c];
    d3 sv = mk3(0.0, 0.0, 0.0), se = sv;
    double cv = 0.0, ce = 0.0;
    for (int i = M.cv_ptr[c] + sub; i < M.cv_ptr[c + 1]; i += kReconLanes) {
      const d3 x = vert(M, M.cv_idx[i]);
      if (dot_x(n, x) + C == 0.0) {
        sv = sv + x;
        cv += 1.0;
      }
    }
    const int fb = cf_begin(M, c), fn = cf_count(M, c);
    for (int q = sub; q < fn; q += kReconLanes) {
      const int e = M.cf_idx[fb + q];
      const int f = e >= 0 ? e : ~e;
      const int b = fv_begin(M, f), k = fv_count(M, f);
      for (int i = 0; i < k; ++i) {
        const int p = M.fv_idx[b + i], r = M.fv_idx[b + (i + 1 == k ? 0 : i + 1)];
        const int from = e >= 0 ? p : r, to = e >= 0 ? r : p;  // outward direction
        if (from > to) continue;
        const d3 xa = vert(M, from), xb = vert(M, to);
        const double sa = dot_x(n, xa) + C, sb = dot_x(n, xb) + C;
        if ((sa > 0.0 && sb < 0.0) || (sa < 0.0 && sb > 0.0)) {
          const double t = sa / (sa - sb);
          se = se + (xa + t * (xb - xa));
          ce += 1.0;
        }
      }
    }
    const double cnt = group_sum(cv) + group_sum(ce);
    const d3 sum = mk3(group_sum(sv.x) + group_sum(se.x), group_sum(sv.y) + group_sum(se.y),
                       group_sum(sv.z) + group_sum(se.z));
    if (sub == 0) {
      const d3 x = cnt > 0.0 ? mk3(sum.x / cnt, sum.y / cnt, sum.z / cnt) : cell_centre(M, c);
      M.lsfir_xc[c] = x.x;
      M.lsfir_xc[nc + c] = x.y;
      M.lsfir_xc[2 * nc + c] = x.z;
    }
  }
}

// One Jacobi rotation of the symmetric 3x3 matrix A (and of the eigenvector
// matrix V) in the (P, Q) plane, zeroing A[P][Q] up to rounding.  An entry
// below 1e-18 of its diagonal pair is set to zero instead (it moves the
// eigenvectors by less than that), so the sweeps end once converged rather
// than chasing rounding.  Compile-time indices keep both matrices in
// registers.
template <int P, int Q>
__device__ inline void jacobi_rotate(double (&A)[3][3], double (&V)[3][3]) {
  const double apq = A[P][Q];
  if (fabs(apq) <= 1e-18 * (fabs(A[P][P]) + fabs(A[Q][Q]))) {
    A[P][Q] = 0.0;
    A[Q][P] = 0.0;
    return;
  }
  const double theta = (A[Q][Q] - A[P][P]) / (2.0 * apq);
  double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));  // the smaller root of t^2 + 2 theta t = 1
  t = theta < 0.0 ? -t : t;
  const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = A[k][P], w = A[k][Q];
    A[k][P] = cs * u - sn * w;
    A[k][Q] = sn * u + cs * w;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = A[P][k], w = A[Q][k];
    A[P][k] = cs * u - sn * w;
    A[Q][k] = sn * u + cs * w;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = V[k][P], w = V[k][Q];
    V[k][P] = cs * u - sn * w;
    V[k][Q] = sn * u + cs * w;
  }
}

// The scatter matrix of one outer pass of LSFIR, a group of kReconLanes
// lanes per interfacial cell; k_lsfir_eig then finds the plane through the cell's PLIC centre x minimising
// sum w_k (n.(x_k - x))^2 over the valid neighbours (interfacial cells
// sharing a vertex whose normals are within 45 degrees), w_k = |x_k - x|^-2.5
// (a neighbour whose centre coincides with x is skipped; with the mesh's
// optional weight floor, |d| is taken as at least 0.05 of the cell's largest
// box extent; evaluated as 1/(d^2 sqrt(sqrt(d^2))), every operation
// correctly rounded).  The lanes load a neighbour each; every lane then
// accumulates the terms in neighbour order through shuffles, the order of a
// serial loop.  In k_lsfir_eig, the normal is the eigenvector of the smallest eigenvalue
// (cyclic Jacobi), turned to agree with the current normal, and is adopted
// when it turns the normal by less than 30/I degrees (cos_turn); with fewer
// than two valid neighbours or a smallest eigenvalue not separated from the
// next, the normal stays.  Results go to lsfir_nn, so every cell reads the
// current normals; the placement pass then moves them over.  After a pass in
// which no normal turned by the tolerance, the later passes do nothing.
__global__ __launch_bounds__(128) void k_lsfir_fit(DevMesh M, int pass, double cos_valid) {
  if (pass > 1 && M.lsfir_turned[pass - 1] == 0) return;
  const int ncell = M.counters[CNT_CELLS];
  const int nc = M.nc;
  const int sub = threadIdx.x & (kReconLanes - 1);
  const int gbase = __lane_id() & ~(kReconLanes - 1);
  const int ngroups = (gridDim.x * blockDim.x) / kReconLanes;
  for (int it = (blockIdx.x * blockDim.x + threadIdx.x) / kReconLanes; it < ncell; it += ngroups) {
    const int c = M.list_cells[it];
    const d3 n = mk3(M.pnx[c], M.pny[c], M.pnz[c]);
    const d3 x = mk3(M.lsfir_xc[c], M.lsfir_xc[nc + c], M.lsfir_xc[2 * nc + c]);
    const double hc = fmax(fmax(M.hix[c] - M.lox[c], M.hiy[c] - M.loy[c]), M.hiz[c] - M.loz[c]);
    const double dmin2 = M.lsfir_cap ? (0.05 * hc) * (0.05 * hc) : 0.0;
    const int nb0 = M.nb_ptr[c], nnb = M.nb_ptr[c + 1] - nb0;
    double A[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    int nvalid = 0;
    for (int r = 0; r < nnb; r += kReconLanes) {
      d3 d = mk3(0.0, 0.0, 0.0);
      double w = 0.0;
      int ok = 0;
      if (r + sub < nnb) {
        const int k = M.nb_idx[nb0 + r + sub];
        if (M.tag_cell[k] == 0 && dot_x(n, mk3(M.pnx[k], M.pny[k], M.pnz[k])) > cos_valid) {
          d = mk3(M.lsfir_xc[k], M.lsfir_xc[nc + k], M.lsfir_xc[2 * nc + k]) - x;
          const double dd = dot_x(d, d);
          if (dd != 0.0) {
            const double dw = fmax(dd, dmin2);
            w = 1.0 / (dw * sqrt(sqrt(dw)));  // |d|^-2.5
            ok = 1;
          }
        }
      }
      const int nq = min(kReconLanes, nnb - r);
      for (int j = 0; j < nq; ++j) {
        if (!__shfl(ok, gbase + j)) continue;  // uniform over the group
        const double dv[3] = {__shfl(d.x, gbase + j), __shfl(d.y, gbase + j), __shfl(d.z, gbase + j)};
        const double wj = __shfl(w, gbase + j);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) A[a][b] = A[a][b] + wj * dv[a] * dv[b];
        ++nvalid;
      }
    }
    if (sub == 0) {  // the matrix and the valid count, for the eigen-solve (a lane per cell)
      double* S6 = M.lsfir_A + 7 * (size_t)it;
      S6[0] = A[0][0]; S6[1] = A[0][1]; S6[2] = A[0][2];
      S6[3] = A[1][1]; S6[4] = A[1][2]; S6[5] = A[2][2];
      S6[6] = (double)nvalid;
    }
  }
}

// The eigen-solve of one LSFIR pass, a lane per interfacial cell (the
// matrices come from k_lsfir_fit): 64 cells' Jacobi iterations run side by
// side in a wavefront.
__global__ void k_lsfir_eig(DevMesh M, int pass, double cos_turn, double cos_stop) {
  if (pass > 1 && M.lsfir_turned[pass - 1] == 0) return;
  const int ncell = M.counters[CNT_CELLS];
  const int nc = M.nc;
  for (int it = grid_stride_start(); it < ncell; it += grid_stride()) {
    const int c = M.list_cells[it];
    const d3 n = mk3(M.pnx[c], M.pny[c], M.pnz[c]);
    const double* S6 = M.lsfir_A + 7 * (size_t)it;
    double A[3][3] = {{S6[0], S6[1], S6[2]}, {S6[1], S6[3], S6[4]}, {S6[2], S6[4], S6[5]}};
    const int nvalid = (int)S6[6];
    d3 e = n;
    if (nvalid >= 2) {
      double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
      for (int sweep = 0; sweep < 64; ++sweep) {
        if (fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]) == 0.0) break;
        jacobi_rotate<0, 1>(A, V);
        jacobi_rotate<0, 2>(A, V);
        jacobi_rotate<1, 2>(A, V);
      }
      // the smallest eigenvalue's column, and the gap to the next
      const double l0 = A[0][0], l1 = A[1][1], l2 = A[2][2];
      const int imin = (l0 <= l1 && l0 <= l2) ? 0 : (l1 <= l2 ? 1 : 2);
      const double lo = imin == 0 ? l0 : (imin == 1 ? l1 : l2);
      const double mid = imin == 0 ? fmin(l1, l2) : (imin == 1 ? fmin(l0, l2) : fmin(l0, l1));
      const double hi = fmax(fmax(l0, l1), l2);
      if (mid - lo > 1e-12 * hi) {
        d3 v = imin == 0 ? mk3(V[0][0], V[1][0], V[2][0]) : (imin == 1 ? mk3(V[0][1], V[1][1], V[2][1])
                                                                         : mk3(V[0][2], V[1][2], V[2][2]));
        const double vn = sqrt(dot_x(v, v));
        v = mk3(v.x / vn, v.y / vn, v.z / vn);
        e = dot_x(v, n) < 0.0 ? mk3(-v.x, -v.y, -v.z) : v;
      }
    }
    const d3 nn = dot_x(e, n) > cos_turn ? e : n;
    M.lsfir_nn[c] = nn.x;
    M.lsfir_nn[nc + c] = nn.y;
    M.lsfir_nn[2 * nc + c] = nn.z;
    if (dot_x(nn, n) < cos_stop) atomicAdd(&M.lsfir_turned[pass], 1);
  }
}

// ============================================================== isosurface-based normals
// (Sec. "Isosurface based interface reconstruction": LLCIR, ELCIR, CLCIR)
constexpr int kIsoLanes = 32;  // a lane per face of the cell
static_assert(kMaxIsoFaces <= kIsoLanes, "a lane per face");

// The isosurface F* = 1/2 of cell c as one polygon, a lane per face of the
// cell.  A vertex is inside when F* >= 1/2; on its face, taken in the cell's
// outward orientation, a lane finds the edge where the walk enters the
// inside and the one where it leaves (0 or 2 crossings; more: no usable
// isosurface).  The polygon is the chain of these segments, each starting at
// the crossing where the previous one ends, from the segment of the cell's
// first face that has one; the chaining broadcasts the current end edge and
// lets the lanes match it by ballot.  On return pos is the lane's place in
// the loop (-1: its face has no segment), p its segment's first point, m the
// loop length; false when min F* < 1/2 < max F* fails, a face has more than
// two crossings or the segments form more than one loop.
__device__ inline bool iso_loop(const DevMesh& M, int c, int sub, int gbase, int& face, int& pos, d3& p, int& m) {
  const int fb = cf_begin(M, c), fn = cf_count(M, c);
  face = -1;
  pos = -1;
  p = mk3(0.0, 0.0, 0.0);
  m = 0;
  int ea = -1, eb = -1, la = -1, lb = -1, ncross = 0;
  double fmn = 2.0, fmx = -1.0;
  if (sub < fn) {
    const int e = M.cf_idx[fb + sub];
    const int f = e >= 0 ? e : ~e;
    face = f;
    const int b = fv_begin(M, f), k = fv_count(M, f);
    for (int i = 0; i < k; ++i) {
      // outward order: as stored for the owner, reversed for the neighbour
      const int ja = e >= 0 ? i : k - 1 - i;
      const int jw = e >= 0 ? (i + 1 == k ? 0 : i + 1) : (i == k - 1 ? k - 1 : k - 2 - i);
      const int a = M.fv_idx[b + ja], w = M.fv_idx[b + jw];
      const double fa = M.Fstar[a], fw = M.Fstar[w];
      fmn = fmin(fmn, fa);
      fmx = fmax(fmx, fa);
      const bool ia = fa >= 0.5, iw = fw >= 0.5;
      if (ia == iw) continue;
      ++ncross;
      if (iw) {
        ea = min(a, w);
        eb = max(a, w);
      } else {
        la = min(a, w);
        lb = max(a, w);
      }
    }
  }
  // min F* < 1/2 < max F* over the cell's vertices (every vertex is on a face)
  double gmn = fmn, gmx = fmx;
#pragma unroll
  for (int o = 1; o < kIsoLanes; o <<= 1) {
    gmn = fmin(gmn, __shfl_xor(gmn, o));
    gmx = fmax(gmx, __shfl_xor(gmx, o));
  }
  const unsigned long long gm = (kIsoLanes == 64 ? ~0ull : ((1ull << kIsoLanes) - 1ull));
  const unsigned long long bad = (__ballot(ncross > 2 || ncross == 1) >> gbase) & gm;
  const unsigned long long valid = (__ballot(ncross == 2) >> gbase) & gm;
  const int nseg = __popcll(valid);
  if (!(gmn < 0.5 && 0.5 < gmx) || bad || nseg < 3) return false;
  const int first = __builtin_ctzll(valid);
  const int fa0 = __shfl(ea, gbase + first), fb0 = __shfl(eb, gbase + first);
  int cur = first;
  for (int n = 0; n < nseg; ++n) {
    if (sub == cur) pos = n;
    const int ca = __shfl(la, gbase + cur), cb = __shfl(lb, gbase + cur);
    if (n == nseg - 1) {
      if (!(ca == fa0 && cb == fb0)) return false;  // the last segment must end where the first starts
      break;
    }
    const unsigned long long mt = (__ballot(ncross == 2 && pos < 0 && ea == ca && eb == cb) >> gbase) & gm;
    if (mt == 0) return false;  // the loop closed early: more than one isosurface
    cur = __builtin_ctzll(mt);
  }
  if (ncross == 2) {
    const double t = (0.5 - M.Fstar[ea]) / (M.Fstar[eb] - M.Fstar[ea]);
    const d3 xa = vert(M, ea), xb = vert(M, eb);
    p = xa + t * (xb - xa);
  }
  m = nseg;
  return true;
}

// Sum over the loop (positions 0..m-1) of cross(r_n - o, r_{n+1} - o), in
// loop order, every lane of the group taking part (r: the lane's ring entry).
__device__ inline d3 iso_fan(d3 o, d3 r, int pos, int m, int gbase) {
  d3 s = mk3(0.0, 0.0, 0.0);
  const unsigned long long gm = (kIsoLanes == 64 ? ~0ull : ((1ull << kIsoLanes) - 1ull));
  int ln = __builtin_ctzll((__ballot(pos == 0) >> gbase) & gm);
  const int l0 = ln;
  for (int n = 0; n < m; ++n) {
    const int lnext = n + 1 < m ? __builtin_ctzll((__ballot(pos == n + 1) >> gbase) & gm) : l0;
    const d3 a = mk3(__shfl(r.x, gbase + ln), __shfl(r.y, gbase + ln), __shfl(r.z, gbase + ln)) - o;
    const d3 b = mk3(__shfl(r.x, gbase + lnext), __shfl(r.y, gbase + lnext), __shfl(r.z, gbase + lnext)) - o;
    s = s + cross_x(a, b);
    ln = lnext;
  }
  return s;
}

// Unit vector of s turned from the loop's side to the fluid (zero for zero s).
__device__ inline d3 iso_unit(d3 s) {
  const double ss = dot_x(s, s);
  if (ss == 0.0) return mk3(0.0, 0.0, 0.0);
  const double inv = -1.0 / sqrt(ss);
  return mk3(s.x * inv, s.y * inv, s.z * inv);
}

// LLCIR, a group per interfacial cell: the isosurface loop, its vertex mean
// g (summed in loop order) and the fan normal about g, turned to the fluid.
// Records whether the cell has a usable isosurface, g and the normal; for
// LLCIR also the normal to place (the cell's current one where there is no
// isosurface).
__global__ __launch_bounds__(128) void k_iso_local(DevMesh M) {
  const int ncell = M.counters[CNT_CELLS];
  const int nc = M.nc;
  const int sub = threadIdx.x & (kIsoLanes - 1);
  const int gbase = __lane_id() & ~(kIsoLanes - 1);
  const int ngroups = (gridDim.x * blockDim.x) / kIsoLanes;
  const unsigned long long gm = (kIsoLanes == 64 ? ~0ull : ((1ull << kIsoLanes) - 1ull));
  for (int it = (blockIdx.x * blockDim.x + threadIdx.x) / kIsoLanes; it < ncell; it += ngroups) {
    const int c = M.list_cells[it];
    int face, pos, m;
    d3 p;
    bool ok = iso_loop(M, c, sub, gbase, face, pos, p, m);
    d3 g = mk3(0.0, 0.0, 0.0), u = g;
    if (ok) {
      for (int n = 0; n < m; ++n) {  // vertex mean in loop order
        const int ln = __builtin_ctzll((__ballot(pos == n) >> gbase) & gm);
        g = g + mk3(__shfl(p.x, gbase + ln), __shfl(p.y, gbase + ln), __shfl(p.z, gbase + ln));
      }
      const double k = (double)m;
      g = mk3(g.x / k, g.y / k, g.z / k);
      u = iso_unit(iso_fan(g, p, pos, m, gbase));
      ok = dot_x(u, u) != 0.0;
    }
    if (sub == 0) {
      M.iso_ok[c] = ok ? 1 : 0;
      M.iso_g[c] = g.x;
      M.iso_g[nc + c] = g.y;
      M.iso_g[2 * nc + c] = g.z;
      M.iso_nl[c] = u.x;
      M.iso_nl[nc + c] = u.y;
      M.iso_nl[2 * nc + c] = u.z;
      if (M.iso_level == 2) {
        const d3 nn = ok ? u : mk3(M.pnx[c], M.pny[c], M.pnz[c]);
        M.lsfir_nn[c] = nn.x;
        M.lsfir_nn[nc + c] = nn.y;
        M.lsfir_nn[2 * nc + c] = nn.z;
      }
    }
  }
}

// ELCIR (clcir = 0) or CLCIR (clcir = 1), a group per interfacial cell with
// an isosurface: the fan about the cell's centre over a ring with one entry
// per polygon edge, the centre of the cell across the face that edge lies on
// (isosurface centres for ELCIR, PLIC centres of the placed ELCIR planes for
// CLCIR), or the edge's first point where that cell has no isosurface.  Kept
// when within 1.2 rad (cos_keep) of the reference normal (LLCIR for ELCIR,
// the placed ELCIR normal for CLCIR); written as the normal to place.
__global__ __launch_bounds__(128) void k_iso_ext(DevMesh M, int clcir, double cos_keep) {
  const int ncell = M.counters[CNT_CELLS];
  const int nc = M.nc;
  const int sub = threadIdx.x & (kIsoLanes - 1);
  const int gbase = __lane_id() & ~(kIsoLanes - 1);
  const int ngroups = (gridDim.x * blockDim.x) / kIsoLanes;
  const double* cen = clcir ? M.lsfir_xc : M.iso_g;
  for (int it = (blockIdx.x * blockDim.x + threadIdx.x) / kIsoLanes; it < ncell; it += ngroups) {
    const int c = M.list_cells[it];
    const d3 cur = mk3(M.pnx[c], M.pny[c], M.pnz[c]);
    d3 nn = cur;
    int face, pos, m;
    d3 p;
    // the same loop k_iso_local found usable (both uniform over the group)
    if (M.iso_ok[c] && iso_loop(M, c, sub, gbase, face, pos, p, m)) {
      d3 r = p;
      if (pos >= 0) {
        const int k = M.owner[face] == c ? M.neigh[face] : M.owner[face];
        if (k >= 0 && M.iso_ok[k]) r = mk3(cen[k], cen[nc + k], cen[2 * nc + k]);
      }
      const d3 o = mk3(cen[c], cen[nc + c], cen[2 * nc + c]);
      const d3 u = iso_unit(iso_fan(o, r, pos, m, gbase));
      const d3 ref = clcir ? cur : mk3(M.iso_nl[c], M.iso_nl[nc + c], M.iso_nl[2 * nc + c]);
      nn = (dot_x(u, u) > 0.0 && dot_x(u, ref) > cos_keep) ? u : ref;
    }
    if (sub == 0) {
      M.lsfir_nn[c] = nn.x;
      M.lsfir_nn[nc + c] = nn.y;
      M.lsfir_nn[2 * nc + c] = nn.z;
    }
  }
}

// ============================================================== update
// Eq. (fnext) with face sums in ascending face order, then the clamp.
constexpr int kUpdateFaces = 6;
__global__ void k_update(DevMesh M, const double* __restrict__ Fin, double* __restrict__ Fout) {
  for (int c = grid_stride_start(); c < M.nc; c += grid_stride()) {
    if (!cell_live(M, c)) continue;
    double VdT = 0.0, VFT = 0.0;
    const int b = cf_begin(M, c), n = cf_count(M, c);  // n >= 4
    // the first kUpdateFaces faces' loads issued together (clamped indices),
    // then summed in face order like the rest
    int eq[kUpdateFaces];
#pragma unroll
    for (int q = 0; q < kUpdateFaces; ++q) eq[q] = M.cf_idx[b + min(q, n - 1)];
    // the cell's own values in the same round trip as its face list (the
    // compiler would otherwise load them after the face sums, a third
    // dependent round trip); the empty asm takes them all at once
    double V = M.V[c], Fc = Fin[c];
    int near = M.flux_near[c];
    static_assert(kUpdateFaces == 6, "the asm below names six face entries");
    asm volatile("" : "+v"(V), "+v"(Fc), "+v"(near), "+v"(eq[0]), "+v"(eq[1]), "+v"(eq[2]), "+v"(eq[3]), "+v"(eq[4]),
                 "+v"(eq[5]));
    // An empty cell none of whose faces carries fluid (every face tag -1, so
    // every V_F is +0): the update gives (0 (1 + h) - 0 / V) / (1 - h) = +0,
    // so its face sums are not gathered.
    if (near == 0 && Fc == 0.0) {
      Fout[c] = 0.0;
      continue;
    }
    double dq[kUpdateFaces], fq[kUpdateFaces];
#pragma unroll
    for (int q = 0; q < kUpdateFaces; ++q) {
      const int fi = eq[q] >= 0 ? eq[q] : ~eq[q];
      dq[q] = M.Vd[fi];
      fq[q] = M.VF[fi];
    }
#pragma unroll
    for (int q = 0; q < kUpdateFaces; ++q) {
      if (q < n) {
        if (eq[q] >= 0) {
          VdT = VdT + dq[q];
          VFT = VFT + fq[q];
        } else {
          VdT = VdT - dq[q];
          VFT = VFT - fq[q];
        }
      }
    }
    // the remaining faces (24 on a cell of the distorted grid) in chunks of
    // kUpdateFaces, each chunk's loads in flight together, summed in face order
    for (int i0 = b + kUpdateFaces; i0 < b + n; i0 += kUpdateFaces) {
      int er[kUpdateFaces];
#pragma unroll
      for (int q = 0; q < kUpdateFaces; ++q) er[q] = M.cf_idx[min(i0 + q, b + n - 1)];
      double dr[kUpdateFaces], fr[kUpdateFaces];
#pragma unroll
      for (int q = 0; q < kUpdateFaces; ++q) {
        const int fi = er[q] >= 0 ? er[q] : ~er[q];
        dr[q] = M.Vd[fi];
        fr[q] = M.VF[fi];
      }
#pragma unroll
      for (int q = 0; q < kUpdateFaces; ++q) {
        if (i0 + q < b + n) {
          if (er[q] >= 0) {
            VdT = VdT + dr[q];
            VFT = VFT + fr[q];
          } else {
            VdT = VdT - dr[q];
            VFT = VFT - fr[q];
          }
        }
      }
    }
    double h = VdT / (2.0 * V);
    double Fn = (Fc * (1.0 + h) - VFT / V) / (1.0 - h);
    Fout[c] = fmin(fmax(Fn, 0.0), 1.0);
  }
}

// ============================================================== refinement initialisation
__device__ inline bool shape_inside(const Shape& s, d3 p) {
  if (s.kind == 0) {
    d3 q = p - mk3(s.a, s.b, s.c);
    return (q.x * q.x + q.y * q.y) + q.z * q.z <= s.d * s.d;
  }
  return dot_x(mk3(s.a, s.b, s.c), p) + s.d >= 0.0;
}

__device__ inline Shape cell_shape(const DevMesh& M, int c, const Shape& sh) {
  return M.prob_shape ? M.prob_shape[problem_of(M, M.cell_pid, c)] : sh;
}

__global__ void k_init_classify(DevMesh M, Shape sh0, double* __restrict__ F) {
  int n = M.nc;
  int stride = grid_stride();
  int base0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  for (int b = base0; b < n; b += stride) {
    int c = b + (threadIdx.x & 63);
    bool refine = false;
    if (c < n) {
      const Shape sh = cell_shape(M, c, sh0);
      bool allin = true, allout = true;
      for (int i = M.cv_ptr[c]; i < M.cv_ptr[c + 1]; ++i) {
        if (shape_inside(sh, vert(M, M.cv_idx[i]))) allout = false;
        else allin = false;
      }
      double val = 0.0;
      if (allin) val = 1.0;
      else if (allout && sh.kind == 1) val = 0.0;
      else if (allout) {
        d3 lo = mk3(M.lox[c], M.loy[c], M.loz[c]), hi = mk3(M.hix[c], M.hiy[c], M.hiz[c]);
        d3 ctr = mk3(sh.a, sh.b, sh.c);
        d3 q = mk3(fmin(fmax(ctr.x, lo.x), hi.x), fmin(fmax(ctr.y, lo.y), hi.y), fmin(fmax(ctr.z, lo.z), hi.z));
        d3 dd = ctr - q;
        if ((dd.x * dd.x + dd.y * dd.y) + dd.z * dd.z > sh.d * sh.d) val = 0.0;
        else refine = true;
      } else refine = true;
      F[c] = val;
    }
    wave_append(refine, c, &M.counters[CNT_REFINE], M.list_cells);
  }
}

// vol(cell ∩ sub-box [∩ half-space])
__device__ inline double cell_subbox_volume(const DevMesh& M, int c, d3 a, d3 b, const Leaf& leaf) {
  if (M.isbox[c]) {
    double v = 0.0;
    for (int k = 0; k < 6; ++k) v += leaf(kuhn_tet(a, b, k));
    return v;
  }
  double acc = 0.0;
  d3 cen = cell_centre(M, c);
  int fb = cf_begin(M, c), fn = cf_count(M, c);
  for (int i = 0; i < fn; ++i) {
    int e = M.cf_idx[fb + i];
    int nt = face_triangle_count(M, e);
    for (int t = 0; t < nt; ++t) {
      d3 t0, t1, t2;
      face_triangle(M, e, t, t0, t1, t2);
      d3 tlo = vmin(vmin(cen, t0), vmin(t1, t2)), thi = vmax(vmax(cen, t0), vmax(t1, t2));
      if (!box_overlap(tlo, thi, a, b)) continue;
      double s6 = det3f(t0 - cen, t1 - cen, t2 - cen);
      if (s6 == 0.0) continue;
      TetCont TC = tet_container(cen, t0, t1, t2);
      double v = 0.0;
      for (int k = 0; k < 6; ++k) {
        double w = clip_volume(kuhn_tet(a, b, k), TC, leaf);
        if (w == -1.0) atomicOr(&M.counters[CNT_ERR], ERR_STACK);
        else v += w;
      }
      acc += s6 > 0.0 ? v : -v;
    }
  }
  return acc;
}

__global__ __launch_bounds__(64) void k_init_refine(DevMesh M, Shape sh0, int ndiv, double* __restrict__ F) {
  int ncell = M.counters[CNT_REFINE];
  const int lane = threadIdx.x;
  for (int it = blockIdx.x; it < ncell; it += gridDim.x) {
    int c = M.list_cells[it];
    const Shape sh = cell_shape(M, c, sh0);
    d3 lo = mk3(M.lox[c], M.loy[c], M.loz[c]), hi = mk3(M.hix[c], M.hiy[c], M.hiz[c]);
    double nd = (double)ndiv;
    d3 hs = mk3((hi.x - lo.x) / nd, (hi.y - lo.y) / nd, (hi.z - lo.z) / nd);
    double acc = 0.0;
    int nsub = ndiv * ndiv * ndiv;
    for (int q = lane; q < nsub; q += 64) {
      int kx = q % ndiv, ky = (q / ndiv) % ndiv, kz = q / (ndiv * ndiv);
      d3 a = mk3(lo.x + (double)kx * hs.x, lo.y + (double)ky * hs.y, lo.z + (double)kz * hs.z);
      d3 b = mk3(lo.x + (double)(kx + 1) * hs.x, lo.y + (double)(ky + 1) * hs.y, lo.z + (double)(kz + 1) * hs.z);
      int nin = 0;
      for (int r = 0; r < 8; ++r) {
        d3 p = mk3((r & 1) ? b.x : a.x, (r & 2) ? b.y : a.y, (r & 4) ? b.z : a.z);
        nin += shape_inside(sh, p) ? 1 : 0;
      }
      if (nin == 0) continue;
      Leaf leaf;
      leaf.useH = false;
      leaf.hn = mk3(0.0, 0.0, 0.0);
      leaf.hd = 0.0;
      if (nin < 8) {
        if (sh.kind == 0) {
          d3 cs = mk3(0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z));
          d3 r = cs - mk3(sh.a, sh.b, sh.c);
          double rl = sqrt(dotf(r, r));
          if (rl > 0.0) {
            leaf.useH = true;
            leaf.hn = mk3(-r.x / rl, -r.y / rl, -r.z / rl);
            leaf.hd = (sh.d - rl) - dotf(leaf.hn, cs);
          }
        } else {
          leaf.useH = true;
          leaf.hn = mk3(sh.a, sh.b, sh.c);
          leaf.hd = sh.d;
        }
      }
      acc += cell_subbox_volume(M, c, a, b, leaf);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) F[c] = acc / M.V[c];
  }
}

// ============================================================== launchers
static inline int blocks_for(long n, int threads, int cap = 1 << 16) {
  long b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

hipError_t launch_zero(int* p, int n, hipStream_t s) {
  k_zero<<<blocks_for(n, 256), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_geometry(const DevMesh& M, hipStream_t s) {
  k_face_geom<<<blocks_for(M.nf, 256), 256, 0, s>>>(M);
  k_cell_geom<<<blocks_for(M.nc, 256), 256, 0, s>>>(M);
  k_node_weights<<<blocks_for(M.nv, 256), 256, 0, s>>>(M);
  return hipGetLastError();
}

#define TIMED(k, launch)          \
  do {                            \
    if (prof) prof->before(k);    \
    launch;                       \
    if (prof) prof->after(k);     \
  } while (0)

hipError_t launch_reconstruct(const DevMesh& M, double* F, const LaunchCfg& L, hipStream_t s, Prof* prof,
                              const LsfirConsts* lsfir) {
  const int st = L.sweep_threads;
  TIMED(K_NODE_TAG, (k_node_tag<<<blocks_for(M.nv, st), st, 0, s>>>(M, F)));
  TIMED(K_CELL_TAG, (k_cell_tag<<<blocks_for(M.nc, st), st, 0, s>>>(M, F)));
  const int rb = blocks_for((long)M.nc * kReconLanes, L.recon_threads, 4096);
  // the first instance launched adds the interfacial cells to the running total
  if (M.any_box) TIMED(K_RECON, (k_recon<true, false><<<rb, L.recon_threads, 0, s>>>(M, F, 1, 0)));
  if (!M.all_box) TIMED(K_RECON, (k_recon<false, false><<<rb, L.recon_threads, 0, s>>>(M, F, M.any_box ? 0 : 1, 0)));
  if (M.iso_level > 0 && lsfir) {
    const int ib = blocks_for((long)M.nc * kIsoLanes, 128, 4096);  // a group of kIsoLanes lanes per cell
    TIMED(K_ISO, (k_iso_local<<<ib, 128, 0, s>>>(M)));
    if (M.iso_level >= 3) TIMED(K_ISO, (k_iso_ext<<<ib, 128, 0, s>>>(M, 0, lsfir->cos_iso)));
    if (M.any_box) TIMED(K_RECON, (k_recon<true, true><<<rb, L.recon_threads, 0, s>>>(M, F, 0, 1)));
    if (!M.all_box) TIMED(K_RECON, (k_recon<false, true><<<rb, L.recon_threads, 0, s>>>(M, F, 0, 1)));
    if (M.iso_level == 4) {
      TIMED(K_PLIC, (k_plic_centres<<<ib, 128, 0, s>>>(M, 0)));
      TIMED(K_ISO, (k_iso_ext<<<ib, 128, 0, s>>>(M, 1, lsfir->cos_iso)));
      if (M.any_box) TIMED(K_RECON, (k_recon<true, true><<<rb, L.recon_threads, 0, s>>>(M, F, 0, 1)));
      if (!M.all_box) TIMED(K_RECON, (k_recon<false, true><<<rb, L.recon_threads, 0, s>>>(M, F, 0, 1)));
    }
  }
  if (M.lsfir_outer > 0 && lsfir) {
    const int lb = blocks_for((long)M.nc * kReconLanes, 128, 4096);  // a group of kReconLanes lanes per cell
    TIMED(K_PLIC, (k_plic_centres<<<lb, 128, 0, s>>>(M, 0)));
    const int eb = blocks_for(M.nc, 64, 1024);
    for (int pass = 1; pass <= M.lsfir_outer; ++pass) {
      TIMED(K_LSFIR_FIT, (k_lsfir_fit<<<lb, 128, 0, s>>>(M, pass, lsfir->cos_valid)));
      TIMED(K_LSFIR_FIT, (k_lsfir_eig<<<eb, 64, 0, s>>>(M, pass, lsfir->cos_turn[pass], lsfir->cos_stop)));
      if (M.any_box) TIMED(K_RECON, (k_recon<true, true><<<rb, L.recon_threads, 0, s>>>(M, F, 0, pass)));
      if (!M.all_box) TIMED(K_RECON, (k_recon<false, true><<<rb, L.recon_threads, 0, s>>>(M, F, 0, pass)));
      if (pass < M.lsfir_outer) TIMED(K_PLIC, (k_plic_centres<<<lb, 128, 0, s>>>(M, pass)));
    }
  }
  return hipGetLastError();
}

hipError_t launch_advect(const DevMesh& M0, const double* uf, const double* uv, double dt, const double* Fin,
                         double* Fout, const LaunchCfg& L, hipStream_t s, Prof* prof, bool reset) {
  DevMesh M = M0;
  if (L.staged_faces > 0 && L.staged_faces < M.poly_cap) M.poly_cap = L.staged_faces;
  if (L.staged_pairs > 0 && L.staged_pairs < M.item_cap)
    M.item_cap = max(kItemRegions, L.staged_pairs - L.staged_pairs % kItemRegions);
  if (L.staged_pairs > 0 && L.staged_pairs < M.unit_cap)
    M.unit_cap = max(kItemRegions, L.staged_pairs - L.staged_pairs % kItemRegions);
  const int st = L.sweep_threads;
  const int pair_grid = kItemRegions * L.pair_blocks_per_region;
  if (reset) k_reset_advect<<<1, 256, 0, s>>>(M);
  TIMED(K_FACE_SWEEP, (k_face_sweep<<<blocks_for(M.nf, st), st, 0, s>>>(M, uf, dt)));
  const int pb = blocks_for(M.nf, 1, L.prep_blocks);
  const double* vel = M.method == kNMFPA ? uf : uv;  // what the flux polyhedra are built from
  const bool p32 = L.prep_lanes == 32;
  if (M.method == kEMFPA) {
    if (p32) TIMED(K_FLUX_PREP, (k_flux_prep<32, kEMFPA><<<pb, kFluxLanes, 0, s>>>(M, vel, dt)));
    else TIMED(K_FLUX_PREP, (k_flux_prep<64, kEMFPA><<<pb, kFluxLanes, 0, s>>>(M, vel, dt)));
  } else if (M.method == kNMFPA) {
    if (p32) TIMED(K_FLUX_PREP, (k_flux_prep<32, kNMFPA><<<pb, kFluxLanes, 0, s>>>(M, vel, dt)));
    else TIMED(K_FLUX_PREP, (k_flux_prep<64, kNMFPA><<<pb, kFluxLanes, 0, s>>>(M, vel, dt)));
  } else {
    if (p32) TIMED(K_FLUX_PREP, (k_flux_prep<32, kFMFPA><<<pb, kFluxLanes, 0, s>>>(M, vel, dt)));
    else TIMED(K_FLUX_PREP, (k_flux_prep<64, kFMFPA><<<pb, kFluxLanes, 0, s>>>(M, vel, dt)));
  }
  if (M.any_box) TIMED(K_FLUX, (k_flux_items_box<<<pair_grid, kItemsBlock, 0, s>>>(M)));
  if (!M.all_box) {
    if (L.filter_lanes == 0) TIMED(K_FLUX_GEN, (k_flux_gen_runs<<<kItemRegions * kRunBlocksPerRegion, kRunBlock, 0, s>>>(M)));
    else if (L.filter_lanes == 8) TIMED(K_FLUX_GEN, (k_flux_gen_filter<8><<<pair_grid, 256, 0, s>>>(M)));
    else if (L.filter_lanes == 16) TIMED(K_FLUX_GEN, (k_flux_gen_filter<16><<<pair_grid, 256, 0, s>>>(M)));
    else if (L.filter_lanes == 64) TIMED(K_FLUX_GEN, (k_flux_gen_filter<64><<<pair_grid, 256, 0, s>>>(M)));
    else TIMED(K_FLUX_GEN, (k_flux_gen_filter<32><<<pair_grid, 256, 0, s>>>(M)));
    if (L.units_rank == 8) TIMED(K_FLUX_GEN_UNITS, (k_flux_gen_units<8><<<pair_grid, kItemsBlock, 0, s>>>(M)));
    else TIMED(K_FLUX_GEN_UNITS, (k_flux_gen_units<4><<<pair_grid, kItemsBlock, 0, s>>>(M)));
    TIMED(K_FLUX_GEN_UDEEP, (k_flux_gen_units_deep<<<1024, 256, 0, s>>>(M)));
    TIMED(K_FLUX_GEN_SUM, (k_flux_gen_sum<<<pair_grid, 256, 0, s>>>(M)));
  }
  TIMED(K_FLUX_DEEP, (k_flux_deep<<<1024, 64, 0, s>>>(M)));
  TIMED(K_FLUX_SUM, (k_flux_sum<<<1024, kFluxLanes, 0, s>>>(M, vel, dt)));
  TIMED(K_UPDATE, (k_update<<<blocks_for(M.nc, st), st, 0, s>>>(M, Fin, Fout)));
  return hipGetLastError();
}

hipError_t launch_tri_cache(const DevMesh& M, hipStream_t s) {
  k_tri_cache<<<blocks_for(M.nc, 256), 256, 0, s>>>(M);
  return hipGetLastError();
}

hipError_t launch_face_tags(const DevMesh& M, hipStream_t s) {
  k_face_tag<<<blocks_for(M.nf, 256), 256, 0, s>>>(M);
  return hipGetLastError();
}

hipError_t launch_init(const DevMesh& M, int kind, const double* p, int ndiv, double* F, hipStream_t s) {
  Shape sh{kind, p[0], p[1], p[2], p[3]};
  k_zero<<<1, 64, 0, s>>>(M.counters + CNT_REFINE, 1);
  k_init_classify<<<blocks_for(M.nc, 256), 256, 0, s>>>(M, sh, F);
  k_init_refine<<<blocks_for(M.nc, 1, 4096), 64, 0, s>>>(M, sh, ndiv, F);
  return hipGetLastError();
}

// ============================================================== static staging
// The flux staging of gvof_advect_step_static lives in this file-scope array
// instead of the mesh's workspace: one copy on each GPU the library runs on,
// held until the process ends.  In host code the array's name is only a
// stand-in for the symbol: its device address comes from hipGetSymbolAddress,
// resolved once per device with that device current, and only that address
// is handed to kernels.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

}  // namespace gvof
