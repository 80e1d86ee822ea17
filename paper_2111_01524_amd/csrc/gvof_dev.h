// Device-side data layout and geometry primitives of the gVOF HIP library.
//
// All arrays are structure-of-arrays in one caller-provided workspace.  The
// whole library is compiled with -ffp-contract=off: expressions that decide
// an integer result (tags, upwind cell, the FMFPA fallback test, box
// detection) are written with plain operators in a fixed order, so they are
// reproducible bit for bit by any IEEE FP64 implementation that evaluates
// them in the same order.  Volume arithmetic, whose result is continuous in
// its inputs, uses explicit fma().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gvof {

// Counters of one region of the pair and unit buffers: fill counters and
// the start of the first reservation that did not fit (INT_MAX: none).
// Faces and pairs reserve their ranges with device-wide atomics on these;
// one cache line per region keeps atomics of different regions apart
// (atomics on one line are serialised).
struct alignas(128) RegionCounters {
  int item_fill, item_okend, unit_fill, unit_okend;
};

struct DevMesh {
  int nv, nf, nc;
  // vertices, faces, connectivity (uploaded once)
  const double *vx, *vy, *vz;
  const int *fv_ptr, *fv_idx, *owner, *neigh;
  const int *cf_ptr, *cf_idx;  // cell -> faces ascending; entry f (cell owns f) or ~f (cell is f's neighbour)
  int fv_stride, cf_stride;    // vertices of every face / faces of every cell when all equal, else 0
  const int *cv_ptr, *cv_idx;  // cell -> distinct vertices ascending
  const int *vc_ptr, *vc_idx;  // vertex -> cells ascending
  double *vc_w, *vc_den;       // node-value weights per vertex-cell entry, and their sum per vertex (set at bind)
  const int *nb_ptr, *nb_idx;  // cell -> vertex-sharing cells ascending (itself excluded)
  // per face (set at bind): where the owner's and the neighbour's lists lie in nb_idx, as
  // (owner's first, owner's count, neighbour's first, neighbour's count); 0, 0 for a boundary face's neighbour
  int4* face_nb;
  const short* cell_np;        // surface triangles of each cell (triangles as they are, polygons fanned)
  // surface triangles of the cells bounded by triangles only, in the order and
  // orientation face_triangle gives them: cell c's are triangles
  // tri_off[c] .. tri_off[c+1]-1 of tri_xyz (9 doubles each); other cells have none
  const int* tri_off;
  double* tri_xyz;
  // geometry (computed on the device at bind)
  double *Sx, *Sy, *Sz, *fcx, *fcy, *fcz;
  double *V, *ccx, *ccy, *ccz, *lox, *loy, *loz, *hix, *hiy, *hiz;
  int8_t* isbox;
  // per-step state
  double* Fstar;
  int8_t *tag_node, *tag_face, *tag_cell;
  // per cell: some face of the cell may carry fluid this step (its face tag
  // is not -1); cleared by the cell tagging, set by the face sweep
  int8_t* flux_near;
  double *pnx, *pny, *pnz, *pC;  // PLIC planes of tag-0 cells
  double *Vd, *VF;
  int* upwind;
  int *list_cells, *list_faces;
  // flux work staging: polyhedron points per listed face, (face, cell, tet) pairs
  double* poly;        // [slot][pts_per_slot][3]: x_0..x_{I-1}, b_0..b_{I-1}, apex, face centre, then (EMFPA) m_0..m_{I-1}
  int pts_per_slot, poly_cap;
  int *item_off, *item_cnt;   // per slot (cnt = -1: face handled by the overflow kernel)
  int *item_slot, *item_cell;  // per pair
  unsigned short* item_tm;     // per pair: flux tet, box cut mask, first-cut width, face vertex count
  double* item_vol;
  int item_cap;
  struct RegionCounters* regions;  // kItemRegions, one cache line each
  // general-cell pairs: surviving (pair, surface tetrahedron) units
  int *item_uoff, *item_ucnt;  // per pair: first unit, unit count (-1: deferred, -2: a box-cell pair)
  int* unit_item;
  unsigned* unit_code;         // surface tetrahedron index, cutting-plane mask << 16, first-cut width bit
  int unit_cap;                // units staged per step at most (kItemRegions regions)
  double* unit_vol;
  int* list_udeep;             // units with four cutting planes
  int* list_over;              // faces not staged (capacity exceeded)
  int* list_deep;              // pairs cut by more planes than the register clip takes
  int* counters;  // [0] tag-0 cells, [1] tag-0 faces, [2] geometry error flags, [3] refine cells
  unsigned long long* totals;  // [0] cells reconstructed, [1] faces with flux polyhedra, [2] staged pairs (cumulative)
  double eps, beta, degen;
  int method;   // flux polyhedra: kFMFPA, kEMFPA or kNMFPA
  // LSFIR (normals refined after LSGIR; lsfir_outer == 0: LSGIR only)
  int lsfir_outer;
  int lsfir_cap;      // weight floor at |d| = 0.05 h (an option, not the paper's weight)
  double* lsfir_xc;   // [3][nc] PLIC centres of the current planes
  double* lsfir_nn;   // [3][nc] fitted normals of the current pass
  double* lsfir_A;    // [7][nc] per listed cell: scatter matrix (upper triangle) and valid-neighbour count
  int* lsfir_turned;  // [kMaxLsfirOuter + 1] cells whose normal turned by the tolerance or more, per pass
  // isosurface-based normals: 0 none, 2 LLCIR, 3 ELCIR, 4 CLCIR (the LSFIR
  // buffers above are shared: lsfir_xc PLIC centres, lsfir_nn normals to place)
  int iso_level;
  double* iso_g;      // [3][nc] isosurface centres
  double* iso_nl;     // [3][nc] LLCIR normals
  int8_t* iso_ok;     // [nc] 1: the interfacial cell has a usable isosurface
  // enclosing box of each problem's vertices ([6][nprob]: lo x y z, hi x y z):
  // flux polyhedron points outside it lie outside the domain (no fluid there)
  // and need no candidate cell
  const double* dom_box;
  int all_box;  // every cell is an axis-aligned box (set at bind)
  int any_box;  // some cell is an axis-aligned box (set at bind)
  // problem partition of a batch (a disjoint union of independent meshes);
  // with nprob == 1 the id arrays are not read
  int nprob;
  const int *vert_pid, *face_pid, *cell_pid;
  // per-problem inputs of a batched step (NULL outside batched calls): time
  // step, and whether the problem advances (inactive problems are left untouched)
  const double* prob_dt;
  const unsigned char* prob_active;
  const struct Shape* prob_shape;  // per-problem body of a batched initialisation
};

// Body of the refinement initialisation: kind 0 sphere (centre a, b, c; radius
// d), kind 1 half-space a x + b y + c z + d >= 0.
struct Shape {
  int kind;
  double a, b, c, d;
};

__device__ inline int problem_of(const DevMesh& M, const int* pid, int i) { return M.nprob > 1 ? pid[i] : 0; }
__device__ inline bool vert_live(const DevMesh& M, int v) {
  return !M.prob_active || M.prob_active[problem_of(M, M.vert_pid, v)] != 0;
}
__device__ inline bool face_live(const DevMesh& M, int f) {
  return !M.prob_active || M.prob_active[problem_of(M, M.face_pid, f)] != 0;
}
__device__ inline bool cell_live(const DevMesh& M, int c) {
  return !M.prob_active || M.prob_active[problem_of(M, M.cell_pid, c)] != 0;
}
// time step of face f: the scalar argument, or its problem's entry in a batched step
__device__ inline double face_dt(const DevMesh& M, int f, double dt) {
  return M.prob_dt ? M.prob_dt[problem_of(M, M.face_pid, f)] : dt;
}

enum { CNT_CELLS = 0, CNT_FACES = 1, CNT_ERR = 2, CNT_REFINE = 3, CNT_ITEMS = 4, CNT_OVER = 5, CNT_DEEP = 6, CNT_UDEEP = 7, CNT_N = 8 };
enum { ERR_APEX = 1, ERR_LEVELS = 2, ERR_STACK = 4, ERR_MESH = 16, ERR_COVER = 32 };

constexpr int kMaxFaceVerts = 8;
// flux polyhedron methods (Secs. "Face-matched", "Edge-matched" and
// "Non-matched flux polyhedron")
constexpr int kFMFPA = 0, kEMFPA = 1, kNMFPA = 2;
constexpr int kMaxLsfirOuter = 32;  // LSFIR outer passes at most
constexpr int kMaxIsoFaces = 32;    // faces of a cell at most for the isosurface reconstructions (a lane each)
constexpr int kItemRegions = 256;
constexpr int kMaxNeighbours = 62;  // vertex-sharing neighbours of one cell
constexpr int kMaxCellVerts = 30;   // distinct vertices of one cell
constexpr int kMaxLevels = 40;      // sorted vertex levels used by the plane-constant search

// ---------------------------------------------------------------- vectors
struct d3 {
  double x, y, z;
};
__host__ __device__ inline d3 mk3(double x, double y, double z) { return d3{x, y, z}; }
__host__ __device__ inline d3 operator+(d3 a, d3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline d3 operator-(d3 a, d3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline d3 operator*(double s, d3 a) { return mk3(s * a.x, s * a.y, s * a.z); }
// exact-order forms (integer decisions depend on them)
__host__ __device__ inline double dot_x(d3 a, d3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__host__ __device__ inline d3 cross_x(d3 a, d3 b) {
  return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// fused forms (continuous results)
__host__ __device__ inline double dotf(d3 a, d3 b) { return fma(a.z, b.z, fma(a.y, b.y, a.x * b.x)); }
__host__ __device__ inline d3 crossf(d3 a, d3 b) {
  return mk3(fma(a.y, b.z, -a.z * b.y), fma(a.z, b.x, -a.x * b.z), fma(a.x, b.y, -a.y * b.x));
}
__host__ __device__ inline double det3f(d3 a, d3 b, d3 c) { return dotf(a, crossf(b, c)); }
__host__ __device__ inline d3 axpy(double t, d3 d, d3 p) { return mk3(fma(t, d.x, p.x), fma(t, d.y, p.y), fma(t, d.z, p.z)); }
__host__ __device__ inline d3 vmin(d3 a, d3 b) { return mk3(fmin(a.x, b.x), fmin(a.y, b.y), fmin(a.z, b.z)); }
__host__ __device__ inline d3 vmax(d3 a, d3 b) { return mk3(fmax(a.x, b.x), fmax(a.y, b.y), fmax(a.z, b.z)); }

__device__ inline d3 vert(const DevMesh& M, int v) { return mk3(M.vx[v], M.vy[v], M.vz[v]); }

// CSR ranges.  When every face has the same vertex count (every cell the same
// face count) the count is kept as a stride and a range costs no load.
__device__ inline int fv_begin(const DevMesh& M, int f) { return M.fv_stride ? f * M.fv_stride : M.fv_ptr[f]; }
__device__ inline int fv_count(const DevMesh& M, int f) {
  return M.fv_stride ? M.fv_stride : M.fv_ptr[f + 1] - M.fv_ptr[f];
}
__device__ inline int cf_begin(const DevMesh& M, int c) { return M.cf_stride ? c * M.cf_stride : M.cf_ptr[c]; }
__device__ inline int cf_count(const DevMesh& M, int c) {
  return M.cf_stride ? M.cf_stride : M.cf_ptr[c + 1] - M.cf_ptr[c];
}
__device__ inline d3 cell_centre(const DevMesh& M, int c) { return mk3(M.ccx[c], M.ccy[c], M.ccz[c]); }

// ---------------------------------------------------------------- tetrahedra and half-spaces
struct Tet {
  d3 p0, p1, p2, p3;
};

__host__ __device__ inline double tet6(const Tet& t) { return det3f(t.p1 - t.p0, t.p2 - t.p0, t.p3 - t.p0); }

__host__ __device__ inline void cswap_desc(double& a, double& b) {
  double hi = fmax(a, b), lo = fmin(a, b);
  a = hi;
  b = lo;
}

// Fraction of a tetrahedron's volume where the affine function with vertex
// values s0..s3 is >= 0.  The fraction depends only on the four values: with
// them sorted a >= b >= c >= d it is, when
//   only a is positive:      a^3 / ((a-b)(a-c)(a-d)),
//   only d is negative:      [abc - d(ab+bc+ca) + d^2(a+b+c)] / ((a-d)(b-d)(c-d)),
//   a, b positive, c, d not: [a^2 b^2 - (c+d) ab (a+b) + cd (a^2+ab+b^2)]
//                              / ((a-c)(a-d)(b-c)(b-d)),
// 1 when d >= 0 and 0 when a <= 0.  The second is 1 - (-d)^3 / ((a-d)(b-d)(c-d))
// and the third the sum of the volumes of the three tetrahedra of the kept
// wedge (vertices a, b and the cut points on ac, ad, bc, bd), each written
// over the common denominator.  In each case every term of the numerator and
// every factor of the denominator is >= 0, so nothing cancels, and the three
// agree where the cases meet.  Computed without branches, with one division.
__host__ __device__ inline double halfspace_fraction(double s0, double s1, double s2, double s3) {
  double a = s0, b = s1, c = s2, d = s3;
  cswap_desc(a, b);
  cswap_desc(c, d);
  cswap_desc(a, c);
  cswap_desc(b, d);
  cswap_desc(b, c);
  const double ab = a * b, apb = a + b;
  const double n1 = (a * a) * a;
  const double d1 = ((a - b) * (a - c)) * (a - d);
  const double n2 = (ab * c - d * fma(c, apb, ab)) + (d * d) * (apb + c);
  const double d2 = ((a - d) * (b - d)) * (c - d);
  const double n3 = (ab * ab - (c + d) * (ab * apb)) + (c * d) * fma(a, a, fma(b, b, ab));
  const double d3 = ((a - c) * (a - d)) * ((b - c) * (b - d));
  const bool one_pos = b <= 0.0, one_neg = c >= 0.0;
  const double num = one_pos ? n1 : (one_neg ? n2 : n3);
  const double den = one_pos ? d1 : (one_neg ? d2 : d3);
  const double f = num / den;
  return d >= 0.0 ? 1.0 : (a <= 0.0 ? 0.0 : f);
}

}  // namespace gvof
