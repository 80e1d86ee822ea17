// C interface of the gVOF HIP library (declarations and contracts: include/gvof.h).
//
// The host side validates the mesh and builds its integer topology (cell ->
// faces, cell -> vertices, vertex -> cells, vertex-sharing neighbours, the
// paper's neigbcell) with counting passes; everything floating point runs in
// the device kernels.  Device memory is one caller-owned workspace carved
// into 256-byte-aligned structure-of-arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gvof.h"
#include "gvof_dev.h"
#include "gvof_launch.h"

using gvof::DevMesh;

// Per-kernel HIP event pairs recorded on the handle's stream.
struct EventProf : gvof::Prof {
  hipStream_t stream = nullptr;
  uint32_t mask = 0;
  struct Rec {
    int k;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t pending = nullptr;
  // A failed event call leaves that launch out of the timings (and out of the
  // launch count); the launch itself is not affected.
  void before(int k) override {
    if (!((mask >> k) & 1u)) return;
    if (hipEventCreate(&pending) != hipSuccess) {
      pending = nullptr;
      return;
    }
    if (hipEventRecord(pending, stream) != hipSuccess) {
      (void)hipEventDestroy(pending);
      pending = nullptr;
    }
  }
  void after(int k) override {
    if (!((mask >> k) & 1u) || !pending) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    if (e && hipEventRecord(e, stream) != hipSuccess) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
    if (e) recs.push_back({k, pending, e});
    else (void)hipEventDestroy(pending);
    pending = nullptr;
  }
  void clear() {
    for (auto& r : recs) {  // nothing to do about a failed destroy
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    recs.clear();
  }
  ~EventProf() override { clear(); }
};

struct gvof_mesh {
  int nv = 0, nf = 0, nc = 0;
  gvof_params p{};
  // host copies / topology (kept until bind)
  std::vector<double> vx, vy, vz;
  std::vector<int> fv_ptr, fv_idx, owner, neigh;
  std::vector<int> cf_ptr, cf_idx, cv_ptr, cv_idx, vc_ptr, vc_idx, nb_ptr, nb_idx;
  std::vector<short> cell_np;  // surface triangles per cell
  std::vector<int> tri_off;    // surface-triangle cache offsets (cells bounded by triangles only)
  int64_t gen_faces = 0;       // faces of cells that are not axis-aligned boxes (the test of the geometry kernel)
  int max_nb = 0;
  // problem partition: problem q owns vertices [voff[q], voff[q+1]), faces
  // [foff[q], foff[q+1]) and cells [coff[q], coff[q+1])
  int nprob = 1;
  std::vector<int> voff, foff, coff;
  gvof::LaunchCfg cfg;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  gvof::Shape* shape_area = nullptr;  // per-problem bodies of a batched initialisation (workspace)
  // device
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int device = -1;  // current device at bind
  DevMesh dm{};
  bool bound = false, reconstructed = false;
  bool advect_state_clear = false;  // a reconstruction cleared the step counters and no advection used them yet
  std::string err;
  EventProf prof;
  gvof::LsfirConsts lsfir{};  // LSFIR thresholds (set at creation)
};

static thread_local std::string g_create_err;

// LSFIR thresholds from the parameters: cos 45 degrees, cos of the stopping
// tolerance, cos(30/I degrees) for each outer pass I.
static void set_lsfir_consts(gvof_mesh* m) {
  const double pi = 3.14159265358979323846;
  m->lsfir.cos_valid = std::sqrt(0.5);
  m->lsfir.cos_stop = std::cos(m->p.lsfir_tol);
  m->lsfir.cos_iso = std::cos(1.2);
  m->lsfir.cos_turn[0] = 1.0;
  for (int i = 1; i <= gvof::kMaxLsfirOuter; ++i) m->lsfir.cos_turn[i] = std::cos((pi / 6.0) / double(i));
}

static int fail(gvof_mesh* m, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (m) m->err = buf;
  else g_create_err = buf;
  return code;
}

#define HIPCHECK(m, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(m, GVOF_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static void cell_counts(gvof_mesh* m);

extern "C" {

void gvof_params_default(gvof_params* p) {
  if (!p) return;
  p->eps = 1e-12;
  p->beta = 1.5;
  p->fmfpa_degen = 1e-12;
  p->flags = GVOF_FLAG_NONE;
  p->lsfir_outer = 4;
  p->lsfir_tol = 1e-3;
}

}  // extern "C"

// fn(begin, end, t) over nt contiguous ranges of [0, n), on worker threads.
template <class Fn>
static int parallel_ranges(int n, Fn fn) {
  const int nt = std::max(1, std::min<int>({(int)std::thread::hardware_concurrency(), 16, n / 4096 + 1}));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back([&, t] { fn((int)((long)n * t / nt), (int)((long)n * (t + 1) / nt), t); });
  fn(0, (int)((long)n / nt), 0);
  for (auto& x : th) x.join();
  return nt;
}

// Per-cell sorted lists built by worker threads over contiguous ranges of
// cells and joined in cell order, so the result is the serial one.  body(c,
// list) fills cell c's list and returns 0, or an error code for the first
// failing cell (the lowest failing cell is reported, as a serial loop would).
template <class Body>
static int per_cell_lists(int nc, std::vector<int>& ptr, std::vector<int>& idx, int& bad_cell, Body body) {
  const int nt = std::max(1, std::min<int>({(int)std::thread::hardware_concurrency(), 16, nc / 4096 + 1}));
  std::vector<std::vector<int>> part(nt);
  std::vector<std::vector<int>> cnt(nt);
  std::vector<int> err(nt, 0), errc(nt, -1);
  auto work = [&](int t) {
    const int c0 = (int)((long)nc * t / nt), c1 = (int)((long)nc * (t + 1) / nt);
    std::vector<int> list;
    cnt[t].reserve(c1 - c0);
    for (int c = c0; c < c1; ++c) {
      list.clear();
      const int e = body(c, list);
      if (e) {
        err[t] = e;
        errc[t] = c;
        return;
      }
      cnt[t].push_back((int)list.size());
      part[t].insert(part[t].end(), list.begin(), list.end());
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  for (int t = 0; t < nt; ++t)
    if (err[t]) {
      bad_cell = errc[t];
      return err[t];
    }
  ptr.assign(nc + 1, 0);
  size_t total = 0;
  for (int t = 0; t < nt; ++t) total += part[t].size();
  idx.clear();
  idx.reserve(total);
  int c = 0;
  for (int t = 0; t < nt; ++t) {
    for (int n : cnt[t]) {
      ptr[c + 1] = ptr[c] + n;
      ++c;
    }
    idx.insert(idx.end(), part[t].begin(), part[t].end());
  }
  return 0;
}

extern "C" {

int gvof_mesh_create(gvof_mesh** out, int32_t nv, const double* vx, const double* vy, const double* vz, int32_t nf,
                     const int32_t* fv_ptr, const int32_t* fv_idx, const int32_t* owner, const int32_t* neigh,
                     int32_t nc, const gvof_params* params) {
  if (!out) return fail(nullptr, GVOF_E_ARG, "out is NULL");
  *out = nullptr;
  if (nv <= 0 || nf <= 0 || nc <= 0) return fail(nullptr, GVOF_E_ARG, "empty mesh (nv=%d nf=%d nc=%d)", nv, nf, nc);
  if (!vx || !vy || !vz || !fv_ptr || !fv_idx || !owner || !neigh) return fail(nullptr, GVOF_E_ARG, "NULL mesh array");
  if (fv_ptr[0] != 0) return fail(nullptr, GVOF_E_MESH, "fv_ptr[0] must be 0");
  for (int f = 0; f < nf; ++f) {
    int k = fv_ptr[f + 1] - fv_ptr[f];
    if (k < 3 || k > GVOF_MAX_FACE_VERTS)
      return fail(nullptr, GVOF_E_MESH, "face %d has %d vertices (3..%d allowed)", f, k, GVOF_MAX_FACE_VERTS);
    if (owner[f] < 0 || owner[f] >= nc) return fail(nullptr, GVOF_E_MESH, "face %d owner %d out of range", f, owner[f]);
    if (neigh[f] < -1 || neigh[f] >= nc || neigh[f] == owner[f])
      return fail(nullptr, GVOF_E_MESH, "face %d neighbour %d invalid", f, neigh[f]);
  }
  long nfv = fv_ptr[nf];
  for (long i = 0; i < nfv; ++i)
    if (fv_idx[i] < 0 || fv_idx[i] >= nv) return fail(nullptr, GVOF_E_MESH, "fv_idx[%ld]=%d out of range", i, fv_idx[i]);
  for (int v = 0; v < nv; ++v)
    if (!std::isfinite(vx[v]) || !std::isfinite(vy[v]) || !std::isfinite(vz[v]))
      return fail(nullptr, GVOF_E_MESH, "vertex %d not finite", v);

  if (params) {
    const uint32_t methods = GVOF_FLAG_EMFPA | GVOF_FLAG_NMFPA;
    const uint32_t recons = GVOF_FLAG_LSFIR | GVOF_FLAG_LLCIR | GVOF_FLAG_ELCIR | GVOF_FLAG_CLCIR;
    const uint32_t known = methods | recons | GVOF_FLAG_LSFIR_CAP;
    if (params->flags & ~known) return fail(nullptr, GVOF_E_ARG, "unknown flags 0x%x", (unsigned)(params->flags & ~known));
    if ((params->flags & methods) == methods)
      return fail(nullptr, GVOF_E_ARG, "GVOF_FLAG_EMFPA and GVOF_FLAG_NMFPA together");
    if (__builtin_popcount(params->flags & recons) > 1)
      return fail(nullptr, GVOF_E_ARG, "more than one reconstruction flag (0x%x)", (unsigned)(params->flags & recons));
    if ((params->flags & GVOF_FLAG_LSFIR) &&
        (params->lsfir_outer < 1 || params->lsfir_outer > GVOF_MAX_LSFIR_OUTER || !(params->lsfir_tol >= 0.0) ||
         !std::isfinite(params->lsfir_tol)))
      return fail(nullptr, GVOF_E_ARG, "lsfir_outer=%d (1..%d) or lsfir_tol=%g (>= 0) invalid", params->lsfir_outer,
                  GVOF_MAX_LSFIR_OUTER, params->lsfir_tol);
  }

  gvof_mesh* m = new gvof_mesh;
  m->nv = nv;
  m->nf = nf;
  m->nc = nc;
  if (params) m->p = *params;
  else gvof_params_default(&m->p);
  set_lsfir_consts(m);
  m->vx.assign(vx, vx + nv);
  m->vy.assign(vy, vy + nv);
  m->vz.assign(vz, vz + nv);
  m->fv_ptr.assign(fv_ptr, fv_ptr + nf + 1);
  m->fv_idx.assign(fv_idx, fv_idx + nfv);
  m->owner.assign(owner, owner + nf);
  m->neigh.assign(neigh, neigh + nf);

  // cell -> faces (ascending face id; ~f marks the neighbour side)
  m->cf_ptr.assign(nc + 1, 0);
  for (int f = 0; f < nf; ++f) {
    m->cf_ptr[owner[f] + 1]++;
    if (neigh[f] >= 0) m->cf_ptr[neigh[f] + 1]++;
  }
  for (int c = 0; c < nc; ++c) m->cf_ptr[c + 1] += m->cf_ptr[c];
  m->cf_idx.assign(m->cf_ptr[nc], 0);
  {
    std::vector<int> fill(m->cf_ptr.begin(), m->cf_ptr.end() - 1);
    for (int f = 0; f < nf; ++f) {
      m->cf_idx[fill[owner[f]]++] = f;
      if (neigh[f] >= 0) m->cf_idx[fill[neigh[f]]++] = ~f;
    }
  }
  for (int c = 0; c < nc; ++c)
    if (m->cf_ptr[c + 1] - m->cf_ptr[c] < 4) {
      delete m;
      return fail(nullptr, GVOF_E_MESH, "cell %d has fewer than 4 faces", c);
    }
  // cell -> distinct vertices (ascending)
  {
    const bool iso = (m->p.flags & (GVOF_FLAG_LLCIR | GVOF_FLAG_ELCIR | GVOF_FLAG_CLCIR)) != 0;
    int bad = -1;
    const int e = per_cell_lists(nc, m->cv_ptr, m->cv_idx, bad, [&](int c, std::vector<int>& tmp) {
      int npoly = 0;
      for (int i = m->cf_ptr[c]; i < m->cf_ptr[c + 1]; ++i) {
        const int e2 = m->cf_idx[i], f = e2 >= 0 ? e2 : ~e2;
        for (int j = fv_ptr[f]; j < fv_ptr[f + 1]; ++j) tmp.push_back(fv_idx[j]);
        if (fv_ptr[f + 1] - fv_ptr[f] > 3) ++npoly;
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      if ((int)tmp.size() > gvof::kMaxCellVerts || (int)tmp.size() + 1 + npoly > gvof::kMaxLevels) return 1;
      if (iso && m->cf_ptr[c + 1] - m->cf_ptr[c] > gvof::kMaxIsoFaces) return 2;
      return 0;
    });
    if (e) {
      const int c = bad;
      int nvc = 0, npoly = 0;
      {
        std::vector<int> tmp;
        for (int i = m->cf_ptr[c]; i < m->cf_ptr[c + 1]; ++i) {
          const int e2 = m->cf_idx[i], f = e2 >= 0 ? e2 : ~e2;
          for (int j = fv_ptr[f]; j < fv_ptr[f + 1]; ++j) tmp.push_back(fv_idx[j]);
          if (fv_ptr[f + 1] - fv_ptr[f] > 3) ++npoly;
        }
        std::sort(tmp.begin(), tmp.end());
        nvc = (int)(std::unique(tmp.begin(), tmp.end()) - tmp.begin());
      }
      const int nfc = m->cf_ptr[c + 1] - m->cf_ptr[c];
      delete m;
      if (e == 1)
        return fail(nullptr, GVOF_E_LIMIT, "cell %d has %d vertices and %d polygon faces (limits %d / %d levels)", c,
                    nvc, npoly, gvof::kMaxCellVerts, gvof::kMaxLevels);
      return fail(nullptr, GVOF_E_LIMIT, "cell %d has %d faces (the isosurface reconstructions take at most %d)", c,
                  nfc, gvof::kMaxIsoFaces);
    }
  }
  // vertex -> cells (ascending)
  m->vc_ptr.assign(nv + 1, 0);
  for (int v : m->cv_idx) m->vc_ptr[v + 1]++;
  for (int v = 0; v < nv; ++v) m->vc_ptr[v + 1] += m->vc_ptr[v];
  m->vc_idx.assign(m->vc_ptr[nv], 0);
  {
    std::vector<int> fill(m->vc_ptr.begin(), m->vc_ptr.end() - 1);
    for (int c = 0; c < nc; ++c)
      for (int i = m->cv_ptr[c]; i < m->cv_ptr[c + 1]; ++i) m->vc_idx[fill[m->cv_idx[i]]++] = c;
  }
  for (int v = 0; v < nv; ++v)
    if (m->vc_ptr[v + 1] == m->vc_ptr[v]) {
      delete m;
      return fail(nullptr, GVOF_E_MESH, "vertex %d belongs to no cell", v);
    }
  // vertex-sharing neighbours (ascending, itself excluded)
  {
    int bad = -1;
    const int e = per_cell_lists(nc, m->nb_ptr, m->nb_idx, bad, [&](int c, std::vector<int>& tmp) {
      for (int i = m->cv_ptr[c]; i < m->cv_ptr[c + 1]; ++i) {
        const int v = m->cv_idx[i];
        for (int j = m->vc_ptr[v]; j < m->vc_ptr[v + 1]; ++j)
          if (m->vc_idx[j] != c) tmp.push_back(m->vc_idx[j]);
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      return (int)tmp.size() > gvof::kMaxNeighbours ? 1 : 0;
    });
    if (e) {
      const int c = bad;
      std::vector<int> tmp;
      for (int i = m->cv_ptr[c]; i < m->cv_ptr[c + 1]; ++i) {
        const int v = m->cv_idx[i];
        for (int j = m->vc_ptr[v]; j < m->vc_ptr[v + 1]; ++j)
          if (m->vc_idx[j] != c) tmp.push_back(m->vc_idx[j]);
      }
      std::sort(tmp.begin(), tmp.end());
      const long n = std::unique(tmp.begin(), tmp.end()) - tmp.begin();
      delete m;
      return fail(nullptr, GVOF_E_LIMIT, "cell %d has %ld vertex neighbours (limit %d)", c, n, gvof::kMaxNeighbours);
    }
    for (int c = 0; c < nc; ++c) m->max_nb = std::max(m->max_nb, m->nb_ptr[c + 1] - m->nb_ptr[c]);
  }
  m->voff = {0, nv};
  m->foff = {0, nf};
  m->coff = {0, nc};
  cell_counts(m);
  *out = m;
  return GVOF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ derived per-cell counts
// Surface triangles per cell (a triangle counts once, a polygon of k vertices
// k times, fanned) and the offsets of the surface-triangle cache, which holds
// the cells bounded by triangles only.
static void cell_counts(gvof_mesh* m) {
  m->cell_np.assign(m->nc, 0);
  m->tri_off.assign(m->nc + 1, 0);
  // per cell: its surface triangles, whether it is bounded by triangles only, and whether it is a box cell
  // (the box test of the geometry kernel: 8 vertices, 6 quadrilateral faces, every vertex a corner of the
  // enclosing box); the counts of general-cell faces are summed per range, then over the ranges
  std::vector<long> gen(16, 0);
  parallel_ranges(m->nc, [&](int c0, int c1, int t) {
    long gf = 0;
    for (int c = c0; c < c1; ++c) {
      int np = 0;
      bool tri_only = true;
      for (int i = m->cf_ptr[c]; i < m->cf_ptr[c + 1]; ++i) {
        int e = m->cf_idx[i], f = e >= 0 ? e : ~e;
        int k = m->fv_ptr[f + 1] - m->fv_ptr[f];
        np += k == 3 ? 1 : k;
        tri_only = tri_only && k == 3;
      }
      m->cell_np[c] = (short)np;
      m->tri_off[c + 1] = tri_only ? np : 0;  // the counts; the offsets follow below
      const int vb = m->cv_ptr[c], vn = m->cv_ptr[c + 1] - vb;
      const int fb = m->cf_ptr[c], fn = m->cf_ptr[c + 1] - fb;
      bool box = vn == 8 && fn == 6;
      for (int i = fb; box && i < fb + fn; ++i) {
        const int e = m->cf_idx[i], f = e >= 0 ? e : ~e;
        box = m->fv_ptr[f + 1] - m->fv_ptr[f] == 4;
      }
      if (box) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int i = vb; i < vb + vn; ++i) {
          const int v = m->cv_idx[i];
          const double p[3] = {m->vx[v], m->vy[v], m->vz[v]};
          for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
          }
        }
        int mask = 0;
        for (int i = vb; box && i < vb + vn; ++i) {
          const int v = m->cv_idx[i];
          const double p[3] = {m->vx[v], m->vy[v], m->vz[v]};
          int bit = 0;
          for (int a = 0; a < 3; ++a) {
            if (p[a] != lo[a] && p[a] != hi[a]) box = false;
            bit |= (p[a] == hi[a] ? 1 : 0) << a;
          }
          mask |= 1 << bit;
        }
        box = box && mask == 255 && lo[0] < hi[0] && lo[1] < hi[1] && lo[2] < hi[2];
      }
      if (!box) gf += fn;
    }
    gen[t] = gf;
  });
  for (int c = 0; c < m->nc; ++c) m->tri_off[c + 1] += m->tri_off[c];
  m->gen_faces = 0;
  for (long g : gen) m->gen_faces += g;
}

// ------------------------------------------------------------------ workspace layout
namespace {
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

size_t carve(gvof_mesh* m, char* base, DevMesh* dm) {
  Carver C{base};
  DevMesh d{};
  size_t nv = m->nv, nf = m->nf, nc = m->nc;
  d.nv = m->nv;
  d.nf = m->nf;
  d.nc = m->nc;
  double* vxyz = C.take<double>(3 * nv);
  d.vx = vxyz;
  d.vy = vxyz ? vxyz + nv : nullptr;
  d.vz = vxyz ? vxyz + 2 * nv : nullptr;
  d.fv_ptr = C.take<int>(nf + 1);
  d.fv_idx = C.take<int>(m->fv_idx.size());
  d.owner = C.take<int>(nf);
  d.neigh = C.take<int>(nf);
  d.cf_ptr = C.take<int>(nc + 1);
  d.cf_idx = C.take<int>(m->cf_idx.size());
  // uniform counts become strides (the kernels then skip the offset loads)
  auto stride_of = [](const std::vector<int>& ptr) {
    const size_t n = ptr.size() - 1;
    const int k = n ? ptr[1] - ptr[0] : 0;
    for (size_t i = 0; i < n; ++i)
      if (ptr[i + 1] - ptr[i] != k) return 0;
    return k;
  };
  d.fv_stride = stride_of(m->fv_ptr);
  d.cf_stride = stride_of(m->cf_ptr);
  d.cv_ptr = C.take<int>(nc + 1);
  d.cv_idx = C.take<int>(m->cv_idx.size());
  d.vc_ptr = C.take<int>(nv + 1);
  d.vc_idx = C.take<int>(m->vc_idx.size());
  d.vc_w = C.take<double>(m->vc_idx.size());
  d.vc_den = C.take<double>(nv);
  d.nb_ptr = C.take<int>(nc + 1);
  d.nb_idx = C.take<int>(std::max<size_t>(m->nb_idx.size(), 1));
  d.face_nb = C.take<int4>(nf);
  d.cell_np = C.take<short>(nc);
  d.tri_off = C.take<int>(nc + 1);
  d.tri_xyz = C.take<double>(9 * std::max<size_t>(m->tri_off.empty() ? 0 : m->tri_off.back(), 1));
  double* S = C.take<double>(3 * nf);
  double* fc = C.take<double>(3 * nf);
  d.Sx = S;
  d.Sy = S ? S + nf : nullptr;
  d.Sz = S ? S + 2 * nf : nullptr;
  d.fcx = fc;
  d.fcy = fc ? fc + nf : nullptr;
  d.fcz = fc ? fc + 2 * nf : nullptr;
  d.V = C.take<double>(nc);
  double* cc = C.take<double>(3 * nc);
  double* lo = C.take<double>(3 * nc);
  double* hi = C.take<double>(3 * nc);
  d.ccx = cc;
  d.ccy = cc ? cc + nc : nullptr;
  d.ccz = cc ? cc + 2 * nc : nullptr;
  d.lox = lo;
  d.loy = lo ? lo + nc : nullptr;
  d.loz = lo ? lo + 2 * nc : nullptr;
  d.hix = hi;
  d.hiy = hi ? hi + nc : nullptr;
  d.hiz = hi ? hi + 2 * nc : nullptr;
  d.isbox = C.take<int8_t>(nc);
  d.Fstar = C.take<double>(nv);
  d.tag_node = C.take<int8_t>(nv);
  d.tag_face = C.take<int8_t>(nf);
  d.tag_cell = C.take<int8_t>(nc);
  d.flux_near = C.take<int8_t>(nc);
  double* pl = C.take<double>(4 * nc);
  d.pnx = pl;
  d.pny = pl ? pl + nc : nullptr;
  d.pnz = pl ? pl + 2 * nc : nullptr;
  d.pC = pl ? pl + 3 * nc : nullptr;
  d.Vd = C.take<double>(nf);
  d.VF = C.take<double>(nf);
  d.upwind = C.take<int>(nf);
  d.list_cells = C.take<int>(nc);
  d.list_faces = C.take<int>(nf);
  {
    int maxI = 3;
    for (size_t f = 0; f < nf; ++f) maxI = std::max(maxI, m->fv_ptr[f + 1] - m->fv_ptr[f]);
    const bool em = (m->p.flags & GVOF_FLAG_EMFPA) != 0;  // (NMFPA: 3I-2 tets, sized as FMFPA)
    // polyhedron points, the face centre, then the EMFPA lateral centres
    d.pts_per_slot = (em ? 3 : 2) * maxI + 2;
    d.poly_cap = (int)std::min<size_t>(nf, std::max<size_t>(65536, nf / 4));
    // EMFPA faces carry 5I flux tets against 3I
    const size_t per_face = em ? 7 : 4, floor_pairs = em ? (size_t(7) << 20) : (size_t(1) << 22);
    d.item_cap = (int)std::min<size_t>(size_t(1) << 30, std::max<size_t>(floor_pairs, per_face * nf));
    d.item_cap -= d.item_cap % gvof::kItemRegions;
    // units: up to about 12 per face of the general cells (6 per cell-face
    // incidence, each face counting for both of its cells) at the most stretched
    // interface of the deformation workload (pairs that do not fit are
    // computed whole by the deferred kernel)
    d.unit_cap = m->gen_faces == 0
                     ? gvof::kItemRegions
                     : (int)std::min<size_t>(size_t(1) << 30, std::max<size_t>(size_t(1) << 22, 8 * (size_t)m->gen_faces));
    d.unit_cap -= d.unit_cap % gvof::kItemRegions;
  }
  d.poly = C.take<double>((size_t)d.poly_cap * d.pts_per_slot * 3);
  d.item_off = C.take<int>(d.poly_cap);
  d.item_cnt = C.take<int>(d.poly_cap);
  d.item_slot = C.take<int>(d.item_cap);
  d.item_cell = C.take<int>(d.item_cap);
  d.item_tm = C.take<unsigned short>(d.item_cap);
  d.item_vol = C.take<double>(d.item_cap);
  d.list_over = C.take<int>(nf);
  d.list_deep = C.take<int>(d.item_cap);
  d.regions = C.take<gvof::RegionCounters>(gvof::kItemRegions);
  d.item_uoff = C.take<int>(d.item_cap);
  d.item_ucnt = C.take<int>(d.item_cap);
  d.unit_item = C.take<int>(d.unit_cap);
  d.unit_code = C.take<unsigned>(d.unit_cap);
  d.unit_vol = C.take<double>(d.unit_cap);
  d.list_udeep = C.take<int>(d.unit_cap);
  d.counters = C.take<int>(gvof::CNT_N);
  if (m->p.flags & (GVOF_FLAG_LLCIR | GVOF_FLAG_ELCIR | GVOF_FLAG_CLCIR)) {
    d.iso_g = C.take<double>(3 * (size_t)nc);
    d.iso_nl = C.take<double>(3 * (size_t)nc);
    d.iso_ok = C.take<int8_t>(nc);
  }
  if (m->p.flags & (GVOF_FLAG_LSFIR | GVOF_FLAG_LLCIR | GVOF_FLAG_ELCIR | GVOF_FLAG_CLCIR)) {
    d.lsfir_xc = C.take<double>(3 * (size_t)nc);
    d.lsfir_nn = C.take<double>(3 * (size_t)nc);
    d.lsfir_A = C.take<double>(7 * (size_t)nc);
    d.lsfir_turned = C.take<int>(gvof::kMaxLsfirOuter + 1);
  }
  d.totals = C.take<unsigned long long>(4);
  d.nprob = m->nprob;
  if (m->nprob > 1) {
    d.vert_pid = C.take<int>(nv);
    d.face_pid = C.take<int>(nf);
    d.cell_pid = C.take<int>(nc);
  }
  gvof::Shape* shp = C.take<gvof::Shape>(m->nprob);
  if (dm) m->shape_area = shp;
  d.dom_box = C.take<double>(6 * (size_t)m->nprob);
  d.eps = m->p.eps;
  d.beta = m->p.beta;
  d.degen = m->p.fmfpa_degen;
  d.method = (m->p.flags & GVOF_FLAG_EMFPA) ? gvof::kEMFPA : (m->p.flags & GVOF_FLAG_NMFPA) ? gvof::kNMFPA : gvof::kFMFPA;
  d.lsfir_outer = (m->p.flags & GVOF_FLAG_LSFIR) ? m->p.lsfir_outer : 0;
  d.lsfir_cap = (m->p.flags & GVOF_FLAG_LSFIR_CAP) ? 1 : 0;
  d.iso_level = (m->p.flags & GVOF_FLAG_LLCIR) ? 2 : (m->p.flags & GVOF_FLAG_ELCIR) ? 3 : (m->p.flags & GVOF_FLAG_CLCIR) ? 4 : 0;
  if (dm) *dm = d;
  return (C.off + 255) & ~size_t(255);
}

// The flux staging of one advection step carved from `bytes` at `base` (the
// static staging array) into d: the region counters, the list of faces left
// to the overflow kernel (one entry per face of the mesh), then polyhedron
// slots, (face, cell, flux tet) pairs and general-cell units, which share the
// rest (slots an eighth; units half when the mesh has general cells).
// Returns the bytes the smallest such layout needs; it fits when that is at
// most `bytes`.
size_t carve_static(const gvof_mesh* m, DevMesh& d, char* base, size_t bytes) {
  constexpr size_t R = gvof::kItemRegions;
  const size_t nf = m->nf;
  const bool gen = m->gen_faces != 0;
  const size_t slot_b = (size_t)d.pts_per_slot * 24 + 8, pair_b = 30, unit_b = 20;
  const size_t fixed = R * sizeof(gvof::RegionCounters) + 4 * nf + 16 * 256;  // alignment slack included
  const size_t min_slots = std::min<size_t>(nf, 256), min_pairs = R * 256, min_units = gen ? R * 256 : R;
  const size_t need = fixed + min_slots * slot_b + min_pairs * pair_b + min_units * unit_b;
  if (need > bytes) return need;
  const size_t rest = bytes - fixed;
  size_t slots = std::max(min_slots, std::min(nf, rest / 8 / slot_b));
  if (rest - slots * slot_b < min_pairs * pair_b + min_units * unit_b) slots = min_slots;
  const size_t left = rest - slots * slot_b;
  const size_t units = gen ? std::max(min_units, ((left - min_pairs * pair_b) / 2 / unit_b) / R * R) : min_units;
  const size_t pairs = ((left - units * unit_b) / pair_b) / R * R;  // >= min_pairs
  Carver C{base};
  d.regions = C.take<gvof::RegionCounters>(R);
  d.list_over = C.take<int>(nf);
  d.poly_cap = (int)slots;
  d.poly = C.take<double>(slots * d.pts_per_slot * 3);
  d.item_off = C.take<int>(slots);
  d.item_cnt = C.take<int>(slots);
  d.item_cap = (int)pairs;
  d.item_slot = C.take<int>(pairs);
  d.item_cell = C.take<int>(pairs);
  d.item_tm = C.take<unsigned short>(pairs);
  d.item_vol = C.take<double>(pairs);
  d.list_deep = C.take<int>(pairs);
  d.item_uoff = C.take<int>(pairs);
  d.item_ucnt = C.take<int>(pairs);
  d.unit_cap = (int)units;
  d.unit_item = C.take<int>(units);
  d.unit_code = C.take<unsigned>(units);
  d.unit_vol = C.take<double>(units);
  d.list_udeep = C.take<int>(units);
  return C.off <= bytes ? need : bytes + 1;
}
}  // namespace

extern "C" {

int gvof_mesh_workspace_bytes(const gvof_mesh* m, size_t* bytes) {
  if (!m || !bytes) return GVOF_E_ARG;
  *bytes = carve(const_cast<gvof_mesh*>(m), nullptr, nullptr);
  return GVOF_OK;
}

int gvof_mesh_bind(gvof_mesh* m, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return GVOF_E_ARG;
  if (!ws) return fail(m, GVOF_E_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(m, GVOF_E_ARG, "workspace must be 256-byte aligned");
  size_t need = carve(m, nullptr, nullptr);
  if (ws_bytes < need) return fail(m, GVOF_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  m->ws = static_cast<char*>(ws);
  m->ws_bytes = ws_bytes;
  m->stream = static_cast<hipStream_t>(stream);
  HIPCHECK(m, hipGetDevice(&m->device));
  carve(m, m->ws, &m->dm);
  DevMesh& d = m->dm;
  hipStream_t s = m->stream;
  size_t nv = m->nv;
  auto up = [&](const void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(const_cast<void*>(dst), src, bytes, hipMemcpyHostToDevice, s);
  };
  HIPCHECK(m, up(d.vx, m->vx.data(), nv * 8));
  HIPCHECK(m, up(d.vy, m->vy.data(), nv * 8));
  HIPCHECK(m, up(d.vz, m->vz.data(), nv * 8));
  HIPCHECK(m, up(d.fv_ptr, m->fv_ptr.data(), m->fv_ptr.size() * 4));
  HIPCHECK(m, up(d.fv_idx, m->fv_idx.data(), m->fv_idx.size() * 4));
  HIPCHECK(m, up(d.owner, m->owner.data(), m->owner.size() * 4));
  HIPCHECK(m, up(d.neigh, m->neigh.data(), m->neigh.size() * 4));
  HIPCHECK(m, up(d.cf_ptr, m->cf_ptr.data(), m->cf_ptr.size() * 4));
  HIPCHECK(m, up(d.cf_idx, m->cf_idx.data(), m->cf_idx.size() * 4));
  HIPCHECK(m, up(d.cv_ptr, m->cv_ptr.data(), m->cv_ptr.size() * 4));
  HIPCHECK(m, up(d.cv_idx, m->cv_idx.data(), m->cv_idx.size() * 4));
  HIPCHECK(m, up(d.vc_ptr, m->vc_ptr.data(), m->vc_ptr.size() * 4));
  HIPCHECK(m, up(d.vc_idx, m->vc_idx.data(), m->vc_idx.size() * 4));
  HIPCHECK(m, up(d.nb_ptr, m->nb_ptr.data(), m->nb_ptr.size() * 4));
  if (!m->nb_idx.empty()) HIPCHECK(m, up(d.nb_idx, m->nb_idx.data(), m->nb_idx.size() * 4));
  HIPCHECK(m, up(d.cell_np, m->cell_np.data(), m->cell_np.size() * sizeof(short)));
  HIPCHECK(m, up(d.tri_off, m->tri_off.data(), m->tri_off.size() * sizeof(int)));
  std::vector<int> pid[3];
  if (m->nprob > 1) {
    const std::vector<int>* offs[3] = {&m->voff, &m->foff, &m->coff};
    int* dst[3] = {const_cast<int*>(d.vert_pid), const_cast<int*>(d.face_pid), const_cast<int*>(d.cell_pid)};
    for (int a = 0; a < 3; ++a) {
      const std::vector<int>& o = *offs[a];
      pid[a].resize(o.back());
      for (int q = 0; q < m->nprob; ++q) std::fill(pid[a].begin() + o[q], pid[a].begin() + o[q + 1], q);
      HIPCHECK(m, up(dst[a], pid[a].data(), pid[a].size() * 4));
    }
  }
  std::vector<double> dom(6 * (size_t)m->nprob);
  for (int q = 0; q < m->nprob; ++q) {
    const int v0 = m->nprob > 1 ? m->voff[q] : 0, v1 = m->nprob > 1 ? m->voff[q + 1] : m->nv;
    double* b = dom.data() + 6 * (size_t)q;
    b[0] = b[3] = m->vx[v0];
    b[1] = b[4] = m->vy[v0];
    b[2] = b[5] = m->vz[v0];
    for (int v = v0 + 1; v < v1; ++v) {
      b[0] = std::min(b[0], m->vx[v]); b[3] = std::max(b[3], m->vx[v]);
      b[1] = std::min(b[1], m->vy[v]); b[4] = std::max(b[4], m->vy[v]);
      b[2] = std::min(b[2], m->vz[v]); b[5] = std::max(b[5], m->vz[v]);
    }
  }
  HIPCHECK(m, up(d.dom_box, dom.data(), dom.size() * 8));
  HIPCHECK(m, gvof::launch_zero(d.counters, gvof::CNT_N, s));
  HIPCHECK(m, gvof::launch_zero(reinterpret_cast<int*>(d.totals), 8, s));
  HIPCHECK(m, gvof::launch_geometry(d, s));
  HIPCHECK(m, gvof::launch_tri_cache(d, s));
  int cnt[gvof::CNT_N];
  HIPCHECK(m, hipMemcpyAsync(cnt, d.counters, sizeof cnt, hipMemcpyDeviceToHost, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  if (cnt[gvof::CNT_ERR] & gvof::ERR_MESH) {
    m->bound = false;
    return fail(m, GVOF_E_MESH, "a cell is not closed or has non-positive volume");
  }
  HIPCHECK(m, gvof::launch_zero(d.counters, gvof::CNT_N, s));
  {
    std::vector<int8_t> box(m->nc);
    HIPCHECK(m, hipMemcpyAsync(box.data(), d.isbox, m->nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(m, hipStreamSynchronize(s));
    d.all_box = std::all_of(box.begin(), box.end(), [](int8_t b) { return b != 0; }) ? 1 : 0;
    d.any_box = std::any_of(box.begin(), box.end(), [](int8_t b) { return b != 0; }) ? 1 : 0;
  }
  HIPCHECK(m, hipStreamSynchronize(s));
  m->bound = true;
  m->reconstructed = false;
  return GVOF_OK;
}

int gvof_set_stream(gvof_mesh* m, void* stream) {
  if (!m) return GVOF_E_ARG;
  m->stream = static_cast<hipStream_t>(stream);
  return GVOF_OK;
}

static void drop_graph(gvof_mesh* m) {  // nothing to do about a failed destroy
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->gexec = nullptr;
  m->graph = nullptr;
}

void gvof_mesh_destroy(gvof_mesh* m) {
  if (!m) return;
  drop_graph(m);
  delete m;
}

int gvof_mesh_sizes(const gvof_mesh* m, int32_t* nv, int32_t* nf, int32_t* nc, int32_t* max_neigh) {
  if (!m) return GVOF_E_ARG;
  if (nv) *nv = m->nv;
  if (nf) *nf = m->nf;
  if (nc) *nc = m->nc;
  if (max_neigh) *max_neigh = m->max_nb;
  return GVOF_OK;
}

static int need_bound(gvof_mesh* m) {
  if (!m) return GVOF_E_ARG;
  if (!m->bound) return fail(m, GVOF_E_ARG, "mesh is not bound to a workspace");
  return GVOF_OK;
}

static int d2d(gvof_mesh* m, void* dst, const void* src, size_t bytes) {
  if (!dst) return GVOF_OK;
  HIPCHECK(m, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, m->stream));
  return GVOF_OK;
}

int gvof_get_geometry(gvof_mesh* m, double* S, double* fc, double* V, double* cc, double* bbmin, double* bbmax,
                      int8_t* isbox) {
  int r = need_bound(m);
  if (r) return r;
  const DevMesh& d = m->dm;
  size_t nf = m->nf, nc = m->nc;
  if ((r = d2d(m, S, d.Sx, 3 * nf * 8))) return r;
  if ((r = d2d(m, fc, d.fcx, 3 * nf * 8))) return r;
  if ((r = d2d(m, V, d.V, nc * 8))) return r;
  if ((r = d2d(m, cc, d.ccx, 3 * nc * 8))) return r;
  if ((r = d2d(m, bbmin, d.lox, 3 * nc * 8))) return r;
  if ((r = d2d(m, bbmax, d.hix, 3 * nc * 8))) return r;
  return d2d(m, isbox, d.isbox, nc);
}

int gvof_init_fraction(gvof_mesh* m, const gvof_shape* shape, int32_t n_div, double* F_out) {
  int r = need_bound(m);
  if (r) return r;
  if (!shape || !F_out) return fail(m, GVOF_E_ARG, "NULL shape or F_out");
  if (n_div < 1 || n_div > 64) return fail(m, GVOF_E_ARG, "n_div=%d outside 1..64", n_div);
  if (shape->kind != GVOF_SHAPE_SPHERE && shape->kind != GVOF_SHAPE_PLANE)
    return fail(m, GVOF_E_ARG, "unknown shape kind %d", shape->kind);
  if (shape->kind == GVOF_SHAPE_SPHERE && !(shape->p[3] > 0.0)) return fail(m, GVOF_E_ARG, "sphere radius <= 0");
  HIPCHECK(m, gvof::launch_init(m->dm, shape->kind, shape->p, n_div, F_out, m->stream));
  return GVOF_OK;
}

int gvof_reconstruct(gvof_mesh* m, double* F, int8_t* cell_tag_out, double* plane_out) {
  int r = need_bound(m);
  if (r) return r;
  if (!F) return fail(m, GVOF_E_ARG, "F is NULL");
  m->prof.stream = m->stream;
  HIPCHECK(m, gvof::launch_reconstruct(m->dm, F, m->cfg, m->stream, m->prof.mask ? &m->prof : nullptr, &m->lsfir));
  m->reconstructed = true;
  m->advect_state_clear = true;
  if ((r = d2d(m, cell_tag_out, m->dm.tag_cell, m->nc))) return r;
  return d2d(m, plane_out, m->dm.pnx, 4 * (size_t)m->nc * 8);
}

int gvof_get_tags(gvof_mesh* m, double* node_value, int8_t* node_tag, int8_t* face_tag, int8_t* cell_tag) {
  int r = need_bound(m);
  if (r) return r;
  if (!m->reconstructed) return fail(m, GVOF_E_ARG, "no reconstruction yet");
  if ((r = d2d(m, node_value, m->dm.Fstar, (size_t)m->nv * 8))) return r;
  if ((r = d2d(m, node_tag, m->dm.tag_node, m->nv))) return r;
  if (face_tag) {
    HIPCHECK(m, gvof::launch_face_tags(m->dm, m->stream));
    if ((r = d2d(m, face_tag, m->dm.tag_face, m->nf))) return r;
  }
  return d2d(m, cell_tag, m->dm.tag_cell, m->nc);
}

int gvof_advect_step(gvof_mesh* m, const double* u_face, const double* u_vert, double dt, const double* F_in,
                     double* F_out, int32_t* upwind_out, double* vd_out, double* vf_out) {
  int r = need_bound(m);
  if (r) return r;
  if (!m->reconstructed) return fail(m, GVOF_E_ARG, "gvof_advect_step needs a preceding gvof_reconstruct");
  const bool nm = (m->p.flags & GVOF_FLAG_NMFPA) != 0;  // NMFPA reads no vertex velocities
  if (!u_face || (!u_vert && !nm) || !F_in || !F_out) return fail(m, GVOF_E_ARG, "NULL array argument");
  if (!std::isfinite(dt)) return fail(m, GVOF_E_ARG, "dt is not finite");
  m->prof.stream = m->stream;
  HIPCHECK(m, gvof::launch_advect(m->dm, u_face, u_vert, dt, F_in, F_out, m->cfg, m->stream,
                                  m->prof.mask ? &m->prof : nullptr, !m->advect_state_clear));
  m->advect_state_clear = false;
  if ((r = d2d(m, upwind_out, m->dm.upwind, (size_t)m->nf * 4))) return r;
  if ((r = d2d(m, vd_out, m->dm.Vd, (size_t)m->nf * 8))) return r;
  return d2d(m, vf_out, m->dm.VF, (size_t)m->nf * 8);
}

int gvof_advect_step_static(gvof_mesh* m, const double* u_face, const double* u_vert, double dt, const double* F_in,
                            double* F_out, int32_t* upwind_out, double* vd_out, double* vf_out) {
  int r = need_bound(m);
  if (r) return r;
  if (!m->reconstructed) return fail(m, GVOF_E_ARG, "gvof_advect_step_static needs a preceding gvof_reconstruct");
  const bool nm = (m->p.flags & GVOF_FLAG_NMFPA) != 0;
  if (!u_face || (!u_vert && !nm) || !F_in || !F_out) return fail(m, GVOF_E_ARG, "NULL array argument");
  if (!std::isfinite(dt)) return fail(m, GVOF_E_ARG, "dt is not finite");
  int dev = -1;
  HIPCHECK(m, hipGetDevice(&dev));
  if (dev != m->device) return fail(m, GVOF_E_ARG, "current device %d is not the mesh's device %d", dev, m->device);
  void* base = nullptr;
  size_t bytes = 0;
  HIPCHECK(m, gvof::static_scratch(&base, &bytes));
  DevMesh d = m->dm;
  const size_t need = carve_static(m, d, static_cast<char*>(base), bytes);
  if (need > bytes)
    return fail(m, GVOF_E_LIMIT, "mesh of %d faces needs %zu bytes of static staging, more than the %zu the library holds "
                "(use gvof_advect_step)", m->nf, need, bytes);
  m->prof.stream = m->stream;
  // the static array keeps the last call's contents: the step clears its region counters first
  HIPCHECK(m, gvof::launch_advect(d, u_face, u_vert, dt, F_in, F_out, m->cfg, m->stream,
                                  m->prof.mask ? &m->prof : nullptr, true));
  m->advect_state_clear = false;
  if ((r = d2d(m, upwind_out, m->dm.upwind, (size_t)m->nf * 4))) return r;
  if ((r = d2d(m, vd_out, m->dm.Vd, (size_t)m->nf * 8))) return r;
  return d2d(m, vf_out, m->dm.VF, (size_t)m->nf * 8);
}

int gvof_interface_counts(gvof_mesh* m, int32_t* n_cells, int32_t* n_faces) {
  int r = need_bound(m);
  if (r) return r;
  int cnt[gvof::CNT_N];
  HIPCHECK(m, hipMemcpyAsync(cnt, m->dm.counters, sizeof cnt, hipMemcpyDeviceToHost, m->stream));
  HIPCHECK(m, hipStreamSynchronize(m->stream));
  if (n_cells) *n_cells = cnt[gvof::CNT_CELLS];
  if (n_faces) *n_faces = cnt[gvof::CNT_FACES];
  return GVOF_OK;
}

int gvof_status(gvof_mesh* m) {
  int r = need_bound(m);
  if (r) return r;
  int cnt[gvof::CNT_N];
  HIPCHECK(m, hipMemcpyAsync(cnt, m->dm.counters, sizeof cnt, hipMemcpyDeviceToHost, m->stream));
  HIPCHECK(m, hipStreamSynchronize(m->stream));
  int e = cnt[gvof::CNT_ERR];
  if (e) {
    return fail(m, GVOF_E_GEOM, "device geometry error flags 0x%x (%s%s%s%s)", e,
                (e & gvof::ERR_APEX) ? "flux-polyhedron apex degenerate " : "",
                (e & gvof::ERR_LEVELS) ? "too many vertex levels " : "",
                (e & gvof::ERR_STACK) ? "clip stack overflow " : "",
                (e & gvof::ERR_COVER) ? "flux polyhedron leaves the cells around its face (time step too large)" : "");
  }
  return GVOF_OK;
}

const char* gvof_last_error(const gvof_mesh* m) { return m ? m->err.c_str() : g_create_err.c_str(); }

int gvof_work_totals(gvof_mesh* m, int64_t* cells, int64_t* faces) {
  int r = need_bound(m);
  if (r) return r;
  unsigned long long t[2];
  HIPCHECK(m, hipMemcpyAsync(t, m->dm.totals, sizeof t, hipMemcpyDeviceToHost, m->stream));
  HIPCHECK(m, hipStreamSynchronize(m->stream));
  if (cells) *cells = (int64_t)t[0];
  if (faces) *faces = (int64_t)t[1];
  return GVOF_OK;
}

int gvof_profile_enable(gvof_mesh* m, uint32_t mask) {
  if (!m) return GVOF_E_ARG;
  m->prof.mask = mask;
  return GVOF_OK;
}

int gvof_profile_read(gvof_mesh* m, int32_t n, double* ms, int64_t* launches) {
  if (!m) return GVOF_E_ARG;
  if (n < 0 || (n > 0 && (!ms || !launches))) return fail(m, GVOF_E_ARG, "bad output arrays");
  HIPCHECK(m, hipStreamSynchronize(m->stream));
  for (int k = 0; k < n; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto& rec : m->prof.recs) {
    float t = 0.f;
    HIPCHECK(m, hipEventElapsedTime(&t, rec.a, rec.b));
    if (rec.k < n) {
      ms[rec.k] += t;
      launches[rec.k] += 1;
    }
  }
  m->prof.clear();
  return GVOF_OK;
}

// ------------------------------------------------------------------ batches
int gvof_batch_create(gvof_mesh** out, int32_t nprob, gvof_mesh* const* parts) {
  if (!out) return fail(nullptr, GVOF_E_ARG, "out is NULL");
  *out = nullptr;
  if (nprob < 1 || !parts) return fail(nullptr, GVOF_E_ARG, "nprob=%d or parts NULL", nprob);
  int64_t nv = 0, nf = 0, nc = 0, nfv = 0, ncf = 0, ncv = 0, nvc = 0, nnb = 0;
  for (int q = 0; q < nprob; ++q) {
    const gvof_mesh* a = parts[q];
    if (!a) return fail(nullptr, GVOF_E_ARG, "part %d is NULL", q);
    if (a->nprob != 1) return fail(nullptr, GVOF_E_ARG, "part %d is itself a batch", q);
    const gvof_params& p0 = parts[0]->p;
    if (a->p.eps != p0.eps || a->p.beta != p0.beta || a->p.fmfpa_degen != p0.fmfpa_degen || a->p.flags != p0.flags ||
        a->p.lsfir_outer != p0.lsfir_outer || a->p.lsfir_tol != p0.lsfir_tol)
      return fail(nullptr, GVOF_E_ARG, "part %d has parameters different from part 0", q);
    nv += a->nv;
    nf += a->nf;
    nc += a->nc;
    nfv += (int64_t)a->fv_idx.size();
    ncf += (int64_t)a->cf_idx.size();
    ncv += (int64_t)a->cv_idx.size();
    nvc += (int64_t)a->vc_idx.size();
    nnb += (int64_t)a->nb_idx.size();
  }
  const int64_t lim = INT32_MAX;
  if (nv > lim || nf > lim || nc > lim || nfv > lim || ncf > lim || ncv > lim || nvc > lim || nnb > lim)
    return fail(nullptr, GVOF_E_LIMIT, "batch exceeds 32-bit indexing (nv=%lld nf=%lld nc=%lld)", (long long)nv,
                (long long)nf, (long long)nc);
  gvof_mesh* m = new gvof_mesh;
  m->p = parts[0]->p;
  set_lsfir_consts(m);
  m->nv = (int)nv;
  m->nf = (int)nf;
  m->nc = (int)nc;
  m->nprob = nprob;
  m->voff.assign(1, 0);
  m->foff.assign(1, 0);
  m->coff.assign(1, 0);
  for (auto* v : {&m->fv_ptr, &m->cf_ptr, &m->cv_ptr, &m->vc_ptr, &m->nb_ptr}) v->assign(1, 0);
  m->vx.reserve(nv);
  m->vy.reserve(nv);
  m->vz.reserve(nv);
  m->fv_idx.reserve(nfv);
  m->owner.reserve(nf);
  m->neigh.reserve(nf);
  m->cf_idx.reserve(ncf);
  m->cv_idx.reserve(ncv);
  m->vc_idx.reserve(nvc);
  m->nb_idx.reserve(nnb);
  // a CSR pointer array continued by a part's (its entries shifted by `base`)
  auto cat_ptr = [](std::vector<int>& dst, const std::vector<int>& src) {
    int base = dst.back();
    for (size_t i = 1; i < src.size(); ++i) dst.push_back(src[i] + base);
  };
  auto cat_idx = [](std::vector<int>& dst, const std::vector<int>& src, int shift) {
    for (int x : src) dst.push_back(x + shift);
  };
  for (int q = 0; q < nprob; ++q) {
    const gvof_mesh* a = parts[q];
    const int vo = m->voff.back(), fo = m->foff.back(), co = m->coff.back();
    m->vx.insert(m->vx.end(), a->vx.begin(), a->vx.end());
    m->vy.insert(m->vy.end(), a->vy.begin(), a->vy.end());
    m->vz.insert(m->vz.end(), a->vz.begin(), a->vz.end());
    cat_ptr(m->fv_ptr, a->fv_ptr);
    cat_idx(m->fv_idx, a->fv_idx, vo);
    cat_idx(m->owner, a->owner, co);
    for (int x : a->neigh) m->neigh.push_back(x >= 0 ? x + co : -1);
    cat_ptr(m->cf_ptr, a->cf_ptr);
    for (int e : a->cf_idx) m->cf_idx.push_back(e >= 0 ? e + fo : ~((~e) + fo));
    cat_ptr(m->cv_ptr, a->cv_ptr);
    cat_idx(m->cv_idx, a->cv_idx, vo);
    cat_ptr(m->vc_ptr, a->vc_ptr);
    cat_idx(m->vc_idx, a->vc_idx, co);
    cat_ptr(m->nb_ptr, a->nb_ptr);
    cat_idx(m->nb_idx, a->nb_idx, co);
    m->max_nb = std::max(m->max_nb, a->max_nb);
    m->voff.push_back(vo + a->nv);
    m->foff.push_back(fo + a->nf);
    m->coff.push_back(co + a->nc);
  }
  cell_counts(m);
  *out = m;
  return GVOF_OK;
}

int gvof_batch_offsets(const gvof_mesh* m, int32_t* nprob, int32_t* vert_off, int32_t* face_off, int32_t* cell_off) {
  if (!m) return GVOF_E_ARG;
  if (nprob) *nprob = m->nprob;
  for (int q = 0; q <= m->nprob; ++q) {
    if (vert_off) vert_off[q] = m->voff[q];
    if (face_off) face_off[q] = m->foff[q];
    if (cell_off) cell_off[q] = m->coff[q];
  }
  return GVOF_OK;
}

int gvof_batch_init_fraction(gvof_mesh* m, const gvof_shape* shapes, int32_t n_div, double* F_out) {
  int r = need_bound(m);
  if (r) return r;
  if (!shapes || !F_out) return fail(m, GVOF_E_ARG, "NULL shapes or F_out");
  if (n_div < 1 || n_div > 64) return fail(m, GVOF_E_ARG, "n_div=%d outside 1..64", n_div);
  std::vector<gvof::Shape> sh(m->nprob);
  for (int q = 0; q < m->nprob; ++q) {
    const gvof_shape& a = shapes[q];
    if (a.kind != GVOF_SHAPE_SPHERE && a.kind != GVOF_SHAPE_PLANE)
      return fail(m, GVOF_E_ARG, "problem %d: unknown shape kind %d", q, a.kind);
    if (a.kind == GVOF_SHAPE_SPHERE && !(a.p[3] > 0.0)) return fail(m, GVOF_E_ARG, "problem %d: radius <= 0", q);
    sh[q] = gvof::Shape{a.kind, a.p[0], a.p[1], a.p[2], a.p[3]};
  }
  HIPCHECK(m, hipMemcpyAsync(m->shape_area, sh.data(), sh.size() * sizeof(gvof::Shape), hipMemcpyHostToDevice,
                             m->stream));
  DevMesh d = m->dm;
  d.prob_shape = m->shape_area;
  const double unused[4] = {0.0, 0.0, 0.0, 1.0};
  HIPCHECK(m, gvof::launch_init(d, GVOF_SHAPE_SPHERE, unused, n_div, F_out, m->stream));
  HIPCHECK(m, hipStreamSynchronize(m->stream));  // the host shape array may go away after return
  return GVOF_OK;
}

static int batch_launch(gvof_mesh* m, const double* uf, const double* uv, const double* dt, const uint8_t* active,
                        double* F, gvof::Prof* prof) {
  DevMesh d = m->dm;
  d.prob_dt = dt;
  d.prob_active = active;
  HIPCHECK(m, gvof::launch_reconstruct(d, F, m->cfg, m->stream, prof, &m->lsfir));
  HIPCHECK(m, gvof::launch_advect(d, uf, uv, 0.0, F, F, m->cfg, m->stream, prof, false));
  m->advect_state_clear = false;
  return GVOF_OK;
}

static int batch_args(gvof_mesh* m, const double* uf, const double* uv, const double* dt, const uint8_t* active,
                      double* F) {
  int r = need_bound(m);
  if (r) return r;
  const bool nm = (m->p.flags & GVOF_FLAG_NMFPA) != 0;  // NMFPA reads no vertex velocities
  if (!uf || (!uv && !nm) || !dt || !active || !F) return fail(m, GVOF_E_ARG, "NULL array argument");
  return GVOF_OK;
}

int gvof_batch_step(gvof_mesh* m, const double* u_face, const double* u_vert, const double* dt,
                    const uint8_t* active, double* F) {
  int r = batch_args(m, u_face, u_vert, dt, active, F);
  if (r) return r;
  m->prof.stream = m->stream;
  if ((r = batch_launch(m, u_face, u_vert, dt, active, F, m->prof.mask ? &m->prof : nullptr))) return r;
  m->reconstructed = true;
  return GVOF_OK;
}

int gvof_graph_capture(gvof_mesh* m, const double* u_face, const double* u_vert, const double* dt,
                       const uint8_t* active, double* F) {
  int r = batch_args(m, u_face, u_vert, dt, active, F);
  if (r) return r;
  if (!m->stream) return fail(m, GVOF_E_ARG, "graph capture needs a stream other than the default stream");
  drop_graph(m);
  HIPCHECK(m, hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
  r = batch_launch(m, u_face, u_vert, dt, active, F, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(m->stream, &g);
  if (r) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return fail(m, GVOF_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  m->graph = g;
  e = hipGraphInstantiate(&m->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(m);
    return fail(m, GVOF_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return GVOF_OK;
}

int gvof_graph_launch(gvof_mesh* m) {
  int r = need_bound(m);
  if (r) return r;
  if (!m->gexec) return fail(m, GVOF_E_ARG, "no captured step (gvof_graph_capture)");
  HIPCHECK(m, hipGraphLaunch(m->gexec, m->stream));
  m->reconstructed = true;
  return GVOF_OK;
}

// ------------------------------------------------------------------ launch shapes
static void cfg_out(const gvof::LaunchCfg& c, gvof_launch_config* o) {
  o->sweep_threads = c.sweep_threads;
  o->recon_threads = c.recon_threads;
  o->prep_blocks = c.prep_blocks;
  o->pair_blocks_per_region = c.pair_blocks_per_region;
  o->filter_lanes = c.filter_lanes;
  o->staged_faces = c.staged_faces;
  o->staged_pairs = c.staged_pairs;
  o->prep_lanes = c.prep_lanes;
  o->units_rank = c.units_rank;
}

int gvof_get_launch_config(const gvof_mesh* m, gvof_launch_config* c) {
  if (!m || !c) return GVOF_E_ARG;
  cfg_out(m->cfg, c);
  return GVOF_OK;
}

int gvof_set_launch_config(gvof_mesh* m, const gvof_launch_config* c) {
  if (!m || !c) return GVOF_E_ARG;
  if (c->sweep_threads < 64 || c->sweep_threads > 1024 || c->sweep_threads % 64)
    return fail(m, GVOF_E_ARG, "sweep_threads=%d (a multiple of 64 in 64..1024)", c->sweep_threads);
  if (c->recon_threads != 64 && c->recon_threads != 128)
    return fail(m, GVOF_E_ARG, "recon_threads=%d (64 or 128)", c->recon_threads);
  if (c->prep_blocks < 1 || c->prep_blocks > (1 << 20))
    return fail(m, GVOF_E_ARG, "prep_blocks=%d (1..2^20)", c->prep_blocks);
  if (c->pair_blocks_per_region < 1 || c->pair_blocks_per_region > 256)
    return fail(m, GVOF_E_ARG, "pair_blocks_per_region=%d (1..256)", c->pair_blocks_per_region);
  if (c->filter_lanes != 0 && c->filter_lanes != 8 && c->filter_lanes != 16 && c->filter_lanes != 32 &&
      c->filter_lanes != 64)
    return fail(m, GVOF_E_ARG, "filter_lanes=%d (0, 8, 16, 32 or 64)", c->filter_lanes);
  if (c->staged_faces < 0) return fail(m, GVOF_E_ARG, "staged_faces=%d (>= 0)", c->staged_faces);
  if (c->staged_pairs < 0) return fail(m, GVOF_E_ARG, "staged_pairs=%d (>= 0)", c->staged_pairs);
  if (c->prep_lanes != 32 && c->prep_lanes != 64)
    return fail(m, GVOF_E_ARG, "prep_lanes=%d (32 or 64)", c->prep_lanes);
  if (c->units_rank != 4 && c->units_rank != 8)
    return fail(m, GVOF_E_ARG, "units_rank=%d (4 or 8)", c->units_rank);
  m->cfg.sweep_threads = c->sweep_threads;
  m->cfg.recon_threads = c->recon_threads;
  m->cfg.prep_blocks = c->prep_blocks;
  m->cfg.pair_blocks_per_region = c->pair_blocks_per_region;
  m->cfg.filter_lanes = c->filter_lanes;
  m->cfg.staged_faces = c->staged_faces;
  m->cfg.staged_pairs = c->staged_pairs;
  m->cfg.prep_lanes = c->prep_lanes;
  m->cfg.units_rank = c->units_rank;
  drop_graph(m);
  return GVOF_OK;
}

int gvof_autotune(gvof_mesh* m, const double* u_face, const double* u_vert, const double* dt, const uint8_t* active,
                  double* F, double* F_save, int32_t reps, gvof_launch_config* best, double* best_ms) {
  int r = batch_args(m, u_face, u_vert, dt, active, F);
  if (r) return r;
  if (!F_save) return fail(m, GVOF_E_ARG, "F_save is NULL");
  if (reps < 1 || reps > 1000) return fail(m, GVOF_E_ARG, "reps=%d outside 1..1000", reps);
  drop_graph(m);
  const size_t fb = (size_t)m->nc * sizeof(double);
  hipStream_t s = m->stream;
  HIPCHECK(m, hipMemcpyAsync(F_save, F, fb, hipMemcpyDeviceToDevice, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(m, hipEventCreate(&e0));
  HIPCHECK(m, hipEventCreate(&e1));
  // time per step of `reps` steps from the saved state (after one untimed step)
  auto timed = [&](const gvof::LaunchCfg& c, double& ms) -> int {
    gvof::LaunchCfg keep = m->cfg;
    m->cfg = c;
    int rr = GVOF_OK;
    HIPCHECK(m, hipMemcpyAsync(F, F_save, fb, hipMemcpyDeviceToDevice, s));
    if ((rr = batch_launch(m, u_face, u_vert, dt, active, F, nullptr))) return rr;
    HIPCHECK(m, hipMemcpyAsync(F, F_save, fb, hipMemcpyDeviceToDevice, s));
    HIPCHECK(m, hipEventRecord(e0, s));
    for (int i = 0; i < reps && !rr; ++i) rr = batch_launch(m, u_face, u_vert, dt, active, F, nullptr);
    HIPCHECK(m, hipEventRecord(e1, s));
    HIPCHECK(m, hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHECK(m, hipEventElapsedTime(&t, e0, e1));
    ms = t / reps;
    m->cfg = keep;
    return rr;
  };
  // the smaller of two timings (a single one is at the mercy of clock changes
  // and other noise of a few percent, the size of the differences sought)
  auto timed2 = [&](const gvof::LaunchCfg& c, double& ms) -> int {
    double a = 0.0, b = 0.0;
    int rr = timed(c, a);
    if (!rr) rr = timed(c, b);
    ms = std::min(a, b);
    return rr;
  };
  gvof::LaunchCfg cur = m->cfg;
  double cur_ms = 0.0;
  if ((r = timed(cur, cur_ms))) return r;  // warm-up, not used
  if ((r = timed2(cur, cur_ms))) return r;
  // coordinate descent over the launch shapes, each with the others fixed
  const int prep[] = {4096, 8192, 16384, 32768};
  const int pbr[] = {4, 8, 16, 32, 64};
  const int lanes[] = {0, 8, 16, 32, 64};
  const int sweep[] = {128, 256, 512, 1024};
  const int recon[] = {64, 128};
  const int plan[] = {64, 32};
  const int urank[] = {4, 8};
  auto sweep_param = [&](int gvof::LaunchCfg::*field, const int* vals, int nvals) -> int {
    for (int i = 0; i < nvals; ++i) {
      if (cur.*field == vals[i]) continue;
      gvof::LaunchCfg c = cur;
      c.*field = vals[i];
      double t = 0.0;
      int rr = timed2(c, t);
      if (rr) return rr;
      if (t < cur_ms) {
        cur = c;
        cur_ms = t;
      }
    }
    return GVOF_OK;
  };
  if ((r = sweep_param(&gvof::LaunchCfg::prep_lanes, plan, 2))) return r;
  if ((r = sweep_param(&gvof::LaunchCfg::prep_blocks, prep, 4))) return r;
  if ((r = sweep_param(&gvof::LaunchCfg::pair_blocks_per_region, pbr, 5))) return r;
  if (!m->dm.all_box && (r = sweep_param(&gvof::LaunchCfg::filter_lanes, lanes, 5))) return r;
  if (!m->dm.all_box && (r = sweep_param(&gvof::LaunchCfg::units_rank, urank, 2))) return r;
  if ((r = sweep_param(&gvof::LaunchCfg::sweep_threads, sweep, 4))) return r;
  if ((r = sweep_param(&gvof::LaunchCfg::recon_threads, recon, 2))) return r;
  m->cfg = cur;
  HIPCHECK(m, hipMemcpyAsync(F, F_save, fb, hipMemcpyDeviceToDevice, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best) cfg_out(cur, best);
  if (best_ms) *best_ms = cur_ms;
  return GVOF_OK;
}

const char* gvof_kernel_name(int32_t k) {
  static const char* names[gvof::K_COUNT] = {"k_node_tag", "k_face_tag", "k_cell_tag", "k_recon",
                                             "k_face_sweep", "k_flux_items_box", "k_update", "k_flux_prep",
                                             "k_flux_sum", "(unused)", "k_flux_gen_filter",
                                             "k_flux_deep", "k_flux_gen_units", "k_flux_gen_sum",
                                             "k_flux_gen_units_deep", "k_lsfir_fit",
                                             "k_plic_centres", "k_iso"};
  return (k >= 0 && k < gvof::K_COUNT) ? names[k] : "";
}

}  // extern "C"
