/*
 * gvof.h -- C interface of the MI355X library for unsplit geometric VOF
 * advection with LSGIR reconstruction and face-matched (FMFPA), edge-matched
 * (EMFPA) or non-matched (NMFPA) flux polyhedra.
 *
 * Method: J. Lopez and J. Hernandez, "gVOF: An open-source package for
 * unsplit geometric volume of fluid methods on arbitrary grids",
 * arXiv 2111.01524.  Section and equation names below refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Status: every int-returning call returns GVOF_OK (0) or a negative
 *    GVOF_E_* code; gvof_last_error() then holds a message.  Argument and mesh
 *    errors are detected on the host before anything is enqueued.  Geometry
 *    failures found on the device (a flux polyhedron whose apex cannot be
 *    placed) set a sticky flag read by gvof_status() after the stream has
 *    been synchronised.
 *  - Memory: arrays passed to gvof_mesh_create are HOST arrays, copied.  All
 *    per-call arrays are DEVICE pointers owned by the caller; the library
 *    never retains them past the call's stream-ordered work.  Vectors are
 *    structure-of-arrays: component k of item i at [k * count + i].
 *  - Device memory of a mesh: the library allocates none.  The caller queries
 *    gvof_mesh_workspace_bytes() and passes one device buffer of at least that
 *    size (256-byte aligned) to gvof_mesh_bind(); it must outlive the mesh.
 *  - Ordering: every call enqueues on the stream given to gvof_mesh_bind()
 *    (or gvof_set_stream()) and returns without synchronising, except the
 *    calls documented as synchronous.  A handle is not thread-safe.
 *  - Precision: all floating point is IEEE FP64.
 */
#ifndef GVOF_H
#define GVOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GVOF_OK = 0,
  GVOF_E_ARG = -1,     /* bad argument (null pointer, size, order of calls) */
  GVOF_E_MESH = -2,    /* mesh fails validation */
  GVOF_E_NOMEM = -3,   /* workspace too small */
  GVOF_E_HIP = -4,     /* HIP runtime error */
  GVOF_E_GEOM = -5,    /* device-detected geometric failure (sticky, see gvof_status) */
  GVOF_E_LIMIT = -6    /* a mesh entity exceeds a compiled-in capacity */
};

/* Flags for gvof_params.flags (any other bit, both method flags, or LSFIR
 * settings out of range: GVOF_E_ARG from gvof_mesh_create); no method flag:
 * FMFPA; no GVOF_FLAG_LSFIR: LSGIR normals */
#define GVOF_FLAG_NONE 0u
/* Flux polyhedra by EMFPA (Sec. "Edge-matched flux polyhedron": vertices moved
 * back along their streak lines, Eq. streak-line2; each lateral face as four
 * triangles about its vertex mean; 3I+1 vertices, 5I+1 faces) instead of
 * FMFPA (Sec. "Face-matched flux polyhedron").  Edge-matched polyhedra of
 * faces with a common vertex share their back vertex and lateral faces to the
 * last bit.  fmfpa_degen is not used with this flag. */
#define GVOF_FLAG_EMFPA 1u
/* Flux polyhedra by NMFPA (Sec. "Non-matched flux polyhedron"): every vertex
 * moved back with the face velocity u_face of the step, so the polyhedron is
 * the face's prism of volume V_d with no adjustment (2I vertices, I+2 faces;
 * neighbouring polyhedra may overlap).  u_vert is not read with this flag.
 * Not together with GVOF_FLAG_EMFPA (GVOF_E_ARG). */
#define GVOF_FLAG_NMFPA 2u
/* Normals by LSFIR (Sec. "Least squares fit interface reconstruction"): after
 * LSGIR, each interfacial cell's normal is refitted as the plane through its
 * PLIC centre (the vertex mean of its PLIC polygon) nearest, in the weighted
 * least-squares sense (w = |dx|^-2.5; a neighbour whose centre coincides
 * with the cell's is skipped), to the PLIC centres of the vertex-sharing
 * interfacial cells whose normals are within 45 degrees; the outer
 * iteration adopts a fit that turns the normal by less than 30/I degrees in
 * pass I, all cells at once, then places the changed planes; at most
 * lsfir_outer passes, stopping early after a pass in which no normal turned
 * by lsfir_tol (radians) or more. */
#define GVOF_FLAG_LSFIR 4u
/* With GVOF_FLAG_LSFIR: the weight of a neighbour whose PLIC centre is closer
 * than 0.05 h (h the largest extent of the cell's box) is taken at
 * |dx| = 0.05 h.  Not part of the paper's method: an option that bounds the
 * weight where two centres nearly coincide and the direction between them
 * is set by rounding.  Ignored without GVOF_FLAG_LSFIR. */
#define GVOF_FLAG_LSFIR_CAP 64u
#define GVOF_MAX_LSFIR_OUTER 32
/* Normals from the isosurface F* = 1/2 of the node values (Sec. "Isosurface
 * based interface reconstruction"; cells without one polygon of it keep
 * LSGIR).  LLCIR: the area-weighted normal of the cell's isosurface polygon
 * fanned about its vertex mean.  ELCIR: the fan about that centre over the
 * isosurface centres of the cells across the polygon's faces, kept within
 * 1.2 rad of LLCIR.  CLCIR: after the ELCIR planes are placed, the same fan
 * over the cells' PLIC centres, kept within 1.2 rad of ELCIR.  Every cell may
 * have at most 32 faces with these flags (GVOF_E_LIMIT).  At most one of the
 * reconstruction flags (LSFIR, LLCIR, ELCIR, CLCIR). */
#define GVOF_FLAG_LLCIR 8u
#define GVOF_FLAG_ELCIR 16u
#define GVOF_FLAG_CLCIR 32u

typedef struct gvof_params {
  double eps;         /* volume-fraction tolerance (Sec. "Interface reconstruction"); 1e-12 as in all tests */
  double beta;        /* LSGIR weight exponent of Eq. (lsgir-beta); 1.5 */
  double fmfpa_degen; /* FMFPA: two lateral planes count as parallel when |d|^2 <= degen |m1|^2 |m2|^2; 1e-12 */
  uint32_t flags;     /* GVOF_FLAG_* */
  int32_t lsfir_outer; /* LSFIR outer passes at most, 1..GVOF_MAX_LSFIR_OUTER; 4, the paper's test setting
                          (Sec. "Test programs and performance analysis") */
  double lsfir_tol;    /* LSFIR stopping angle (rad), >= 0 (0: stop only when no normal moved); 1e-3, the
                          paper's test setting */
} gvof_params;

/* Fills the defaults quoted above. */
void gvof_params_default(gvof_params* p);

typedef struct gvof_mesh gvof_mesh;

/*
 * Mesh (Sec. "Grid construction"): nv vertices; nf planar polygonal faces,
 * face f having vertices fv_idx[fv_ptr[f] .. fv_ptr[f+1]-1] ordered
 * counter-clockwise seen from outside its owner cell; owner[f] in [0, nc),
 * neigh[f] in [0, nc) or -1 on the domain boundary.  Faces with 3 vertices
 * are used as they are; larger polygons are fanned from their vertex mean.
 *
 * Validates (ranges, >= 3 and <= GVOF_MAX_FACE_VERTS vertices per face,
 * owner != neigh) and builds the topology on the host: cell -> face lists,
 * cell -> vertex lists, vertex -> cell lists and the vertex-sharing neighbour
 * list of every cell (the paper's neigbcell).  Closedness and positive
 * volumes are checked on the device by gvof_mesh_bind.  All arrays are
 * host memory, copied; on failure *out is NULL and the status says why.
 */
#define GVOF_MAX_FACE_VERTS 8
int gvof_mesh_create(gvof_mesh** out, int32_t nv, const double* vx, const double* vy, const double* vz,
                     int32_t nf, const int32_t* fv_ptr, const int32_t* fv_idx, const int32_t* owner,
                     const int32_t* neigh, int32_t nc, const gvof_params* params);

/* Bytes of device workspace the mesh needs (geometry, topology, per-step state). */
int gvof_mesh_workspace_bytes(const gvof_mesh* m, size_t* bytes);

/*
 * Uploads the mesh into dev_workspace (device pointer, >= workspace bytes,
 * 256-byte aligned), computes the grid geometry on the device (the paper's
 * compgrid: face area vectors and vertex means, cell volumes, vertex means,
 * enclosing boxes) and checks that every cell is closed and has positive
 * volume.  `stream` is a hipStream_t (NULL = default stream).  Synchronous.
 */
int gvof_mesh_bind(gvof_mesh* m, void* dev_workspace, size_t ws_bytes, void* stream);

/* Changes the stream later calls enqueue on. */
int gvof_set_stream(gvof_mesh* m, void* stream);

void gvof_mesh_destroy(gvof_mesh* m);

/* Counts of the mesh: nv, nf, nc, and the largest vertex-neighbour list. */
int gvof_mesh_sizes(const gvof_mesh* m, int32_t* nv, int32_t* nf, int32_t* nc, int32_t* max_neigh);

/*
 * Copies the device-computed geometry into caller device buffers (any may be
 * NULL): S (3 x nf) face area vectors = 1/2 sum (x_i - c) x (x_{i+1} - c),
 * fc (3 x nf) face vertex means, V (nc) cell volumes, cc (3 x nc) cell vertex
 * means, bbmin/bbmax (3 x nc) enclosing boxes, isbox (nc) 1 for axis-aligned
 * box cells.
 */
int gvof_get_geometry(gvof_mesh* m, double* S, double* fc, double* V, double* cc, double* bbmin,
                      double* bbmax, int8_t* isbox);

/*
 * Refinement initialisation (Sec. "Fluid volume fraction initialization"):
 * F_out (device, nc) receives the fraction of every cell inside the body.
 * Each cell's enclosing box is split into n_div^3 sub-boxes; a sub-box with
 * all 8 corners inside counts its part inside the cell whole, one with none
 * inside counts nothing, and a mixed one counts its part inside the cell and
 * on the inner side of the body's tangent plane at the sub-box centre.
 * Cells whose vertices are all inside are full; cells whose vertices are all
 * outside and whose box misses the body are empty.
 */
typedef struct gvof_shape {
  int32_t kind;     /* GVOF_SHAPE_SPHERE: p = (cx, cy, cz, r); GVOF_SHAPE_PLANE: inside n.x + C >= 0, p = (nx, ny, nz, C) */
  double p[4];
} gvof_shape;
#define GVOF_SHAPE_SPHERE 0
#define GVOF_SHAPE_PLANE 1
int gvof_init_fraction(gvof_mesh* m, const gvof_shape* shape, int32_t n_div, double* F_out);

/*
 * Reconstruction (Sec. "Interface reconstruction", Sec. "Grid tagging"):
 *  1. node values F* by inverse-distance weighting (weights 1/|x_v - x_c|^2)
 *     of the cells sharing the node, node tags, face tags, cell tags, all in
 *     {-1, 0, 1} with tolerance eps;
 *  2. cut-off of F in place: F < eps -> 0, F > 1 - eps -> 1;
 *  3. for every cell tagged 0: LSGIR normal n = grad F / |grad F| with grad F
 *     the weighted least-squares solution of Eqs. (lsgir1), (lsgir2),
 *     (lsgir-beta) over the vertex-sharing neighbours, and the constant C of
 *     the PLIC plane n.x + C = 0 (Eq. plic-eq), fluid on n.x + C >= 0, such
 *     that the fluid part of the cell has volume F V (for F > 1/2 solved on
 *     the empty part, (1 - F) V, the same plane);
 *  4. with GVOF_FLAG_LSFIR, GVOF_FLAG_LLCIR, GVOF_FLAG_ELCIR or
 *     GVOF_FLAG_CLCIR in the mesh's parameters, the normals are then replaced
 *     as that flag describes and the changed planes placed again as in 3.
 * F_inout (device, nc) in: fractions, out: cut-off fractions.  Optional
 * device outputs (may be NULL): cell_tag_out (nc), plane_out (4 x nc: nx, ny,
 * nz, C; zero for cells not tagged 0).  The tags and planes are also kept in
 * the workspace for the next gvof_advect_step.
 */
int gvof_reconstruct(gvof_mesh* m, double* F_inout, int8_t* cell_tag_out, double* plane_out);

/*
 * Tags and node values of the last reconstruction into caller device buffers
 * (any may be NULL): node_value (nv), node_tag (nv), face_tag (nf), cell_tag (nc).
 */
int gvof_get_tags(gvof_mesh* m, double* node_value, int8_t* node_tag, int8_t* face_tag, int8_t* cell_tag);

/*
 * Advection step (Sec. "Fluid advected through cell faces"):
 *  - V_d = dt u_f . S_f per face (Eq. a-donacion, u_f the face velocity at
 *    t^{n+1/2}); upwind cell = owner if V_d >= 0 else neighbour (-1 outside);
 *  - V_F per face: 0 for faces tagged -1 and for inflow boundary faces; V_d
 *    for faces tagged 1; otherwise the signed fluid volume of the face's flux
 *    polyhedron (FMFPA, or EMFPA / NMFPA by the mesh's flags) built from the
 *    vertex velocities u_vert (NMFPA: from u_face), truncated by the PLIC
 *    half-spaces of the cells it overlaps (candidates: the owner, the
 *    neighbour and every cell sharing a vertex with either);
 *  - F_out = Eq. (fnext) with the face sums over each cell, clamped to [0, 1].
 * u_face (3 x nf), u_vert (3 x nv; may be NULL with GVOF_FLAG_NMFPA), F_in,
 * F_out (nc): device.  F_out may alias
 * F_in.  Optional device outputs (may be NULL): upwind_out (nf, int32),
 * vd_out (nf), vf_out (nf).  Needs a preceding gvof_reconstruct (it uses the
 * tags and planes made there).  dt must be finite; a negative dt advects
 * with the velocity reversed.
 */
int gvof_advect_step(gvof_mesh* m, const double* u_face, const double* u_vert, double dt, const double* F_in,
                     double* F_out, int32_t* upwind_out, double* vd_out, double* vf_out);

/*
 * gvof_advect_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, the same results bit for bit, the same errors.  The
 * step's flux staging (polyhedron slots, (face, cell, flux tetrahedron)
 * pairs, general-cell units, the overflow and deferred lists and the region
 * counters) lives in a 16 MiB device array inside the library instead of the
 * mesh's workspace: one array on each GPU the library runs on, held until the
 * process ends.  Faces and pairs that do not fit it are computed by the
 * overflow and deferred kernels, with the same values.  Each call clears the
 * array's counters first; every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads) race.  The
 * current device must be the mesh's (the current device at gvof_mesh_bind;
 * GVOF_E_ARG otherwise).  A mesh whose overflow list does not fit the array
 * (more than about 3.4 million faces) is rejected with GVOF_E_LIMIT before
 * anything is enqueued.  Calls no hipMalloc, hipFree or allocating routine.
 */
int gvof_advect_step_static(gvof_mesh* m, const double* u_face, const double* u_vert, double dt,
                            const double* F_in, double* F_out, int32_t* upwind_out, double* vd_out,
                            double* vf_out);

/*
 * Number of interfacial cells of the last reconstruction and of faces needing
 * flux polyhedra in the last advection (0 when a reconstruction came after
 * it).  Synchronous (reads two device counters).
 */
int gvof_interface_counts(gvof_mesh* m, int32_t* n_cells, int32_t* n_faces);

/*
 * Cumulative work counters since bind (device-side, no synchronisation per
 * step): interfacial cells reconstructed and faces given flux polyhedra,
 * summed over every call.  Synchronous read.
 */
int gvof_work_totals(gvof_mesh* m, int64_t* cells, int64_t* faces);

/*
 * Kernel timing instrumentation (not part of the method).  While enabled, the
 * kernels selected by `mask` (bit k = kernel k of gvof_kernel_name) are
 * bracketed by HIP events recorded on the handle's stream.  gvof_profile_read
 * synchronises, writes for every kernel k < n the summed milliseconds and the
 * number of timed launches, and clears the record.
 */
#define GVOF_NUM_KERNELS 18
int gvof_profile_enable(gvof_mesh* m, uint32_t mask);
int gvof_profile_read(gvof_mesh* m, int32_t n, double* ms, int64_t* launches);
const char* gvof_kernel_name(int32_t k);

/*
 * Batches of independent problems.  The method advances every problem on its
 * own (Sec. "Problem statement"); a batch only lets one pass of each kernel
 * serve many problems, over flat work lists that span all of them.
 *
 * gvof_batch_create makes a new, unbound handle whose mesh is the disjoint
 * union of `nprob` handles made by gvof_mesh_create (bound or not; they are
 * copied and may be destroyed afterwards).  Problem q owns the vertex, face
 * and cell ranges reported by gvof_batch_offsets, in part order; each part's
 * own numbering is kept within its range, so per-problem results are
 * bit-identical to those of the part alone.  All parts must have the same
 * gvof_params.  Indices must fit 32 bits (GVOF_E_LIMIT otherwise).  Every
 * single-problem call works on a batch too, treating it as one problem.
 */
int gvof_batch_create(gvof_mesh** out, int32_t nprob, gvof_mesh* const* parts);

/* Host arrays of nprob+1 entries each (any may be NULL): range starts of each problem, then the totals. */
int gvof_batch_offsets(const gvof_mesh* m, int32_t* nprob, int32_t* vert_off, int32_t* face_off, int32_t* cell_off);

/*
 * gvof_init_fraction with one body per problem: shapes is a HOST array of
 * nprob entries.  Synchronous.
 */
int gvof_batch_init_fraction(gvof_mesh* m, const gvof_shape* shapes, int32_t n_div, double* F_out);

/*
 * One step of every active problem: gvof_reconstruct followed by
 * gvof_advect_step, in place on F (device, nc).  dt (device, nprob doubles)
 * holds each problem's time step; active (device, nprob bytes) selects the
 * problems that advance: the vertices, faces and cells of a problem with
 * active[q] == 0 are neither read for work nor written, so its F stays as it
 * is.  u_face (3 x nf) and u_vert (3 x nv) as in gvof_advect_step, over the
 * batch's numbering.  dt and active are read on the device when the step
 * runs, so a captured step (gvof_graph_capture) follows their current
 * contents.
 */
int gvof_batch_step(gvof_mesh* m, const double* u_face, const double* u_vert, const double* dt,
                    const uint8_t* active, double* F);

/*
 * Captures one gvof_batch_step with these device pointers into a HIP graph
 * owned by the handle (replacing any previous one), and replays it on the
 * handle's stream, which must not be the default stream.  The pointers are
 * baked into the graph: the arrays must stay allocated while it is used.  The
 * graph is dropped by gvof_set_launch_config, gvof_autotune and
 * gvof_mesh_destroy.  The captured step contains kernels only (no memset or
 * copy nodes).
 */
int gvof_graph_capture(gvof_mesh* m, const double* u_face, const double* u_vert, const double* dt,
                       const uint8_t* active, double* F);
int gvof_graph_launch(gvof_mesh* m);

/*
 * Launch shapes of the step's kernels.  None of them changes any result (every
 * sum has a fixed order whatever the mapping); they change only the time.
 *   sweep_threads           block size of the vertex / face / cell sweeps (multiple of 64, 64..1024)
 *   recon_threads           block size of the reconstruction kernel (64 or 128)
 *   prep_blocks             grid of the flux-polyhedron staging kernel, blocks of one wavefront (1..2^20)
 *   pair_blocks_per_region  blocks serving each of the 256 regions of the pair buffer (1..256) in the box-cell
 *                           truncation, the per-pair general-cell filter, the unit kernel and the sums
 *   filter_lanes            general-cell filter: 0 takes each run of a face's pairs with one cell together
 *                           (a group of 32 lanes per run, two groups per one-wavefront block, over a grid
 *                           of its own; the default); 8, 16, 32, 64 give each (face, cell, flux
 *                           tetrahedron) pair that many lanes.  Every choice gives the same units.
 *   staged_faces            most faces whose flux work is staged per step (0: as many as the workspace
 *                           holds); the others are computed whole by the overflow kernel, with the same
 *                           values.  Not tuned by gvof_autotune.
 *   staged_pairs            most (face, cell, flux tetrahedron) pairs, and most general-cell units, staged per
 *                           step (0: as many as the workspace holds, else rounded down to a multiple of 256,
 *                           at least 256); faces and pairs that do not fit are computed by the overflow and
 *                           deferred kernels, with the same values.  Not tuned by gvof_autotune.
 *   prep_lanes              lanes per face in the staging kernel (64: one face per wavefront, 32: two)
 *   units_rank              general-cell units ranked by their work together per thread of the unit kernel
 *                           (4 or 8: blocks of 256 threads rank 1024 or 2048 units at a time)
 */
typedef struct gvof_launch_config {
  int32_t sweep_threads;
  int32_t recon_threads;
  int32_t prep_blocks;
  int32_t pair_blocks_per_region;
  int32_t filter_lanes;
  int32_t staged_faces;
  int32_t staged_pairs;
  int32_t prep_lanes;
  int32_t units_rank;
} gvof_launch_config;
int gvof_get_launch_config(const gvof_mesh* m, gvof_launch_config* c);
int gvof_set_launch_config(gvof_mesh* m, const gvof_launch_config* c);

/*
 * Chooses the launch shapes for this mesh and these inputs by measurement:
 * coordinate descent over the values of each field, every candidate timed
 * twice with HIP events over `reps` batched steps (1..1000) from the same
 * state, the smaller time counting (after one untimed warm-up timing).
 * F (device, nc) is saved into F_save (device, nc, caller scratch) first and
 * restored at the end, so F is unchanged on return.  Sets the handle's launch
 * shapes to the best found and reports them and their time per step (either
 * output may be NULL).  Synchronous.
 */
int gvof_autotune(gvof_mesh* m, const double* u_face, const double* u_vert, const double* dt, const uint8_t* active,
                  double* F, double* F_save, int32_t reps, gvof_launch_config* best, double* best_ms);

/* Synchronises the stream and returns GVOF_OK or the sticky GVOF_E_GEOM. */
int gvof_status(gvof_mesh* m);

/* Message of the last error on this handle (or of the last failed create when m is NULL). */
const char* gvof_last_error(const gvof_mesh* m);

#ifdef __cplusplus
}
#endif
#endif /* GVOF_H */
