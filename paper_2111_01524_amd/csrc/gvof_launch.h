// Host-side launchers of the gVOF kernels (defined in gvof_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gvof_dev.h"

namespace gvof {
// (K_FLUX_OVER keeps its index but is no longer a launch of its own: the
// overflow faces are computed by the k_flux_sum launch)
enum KernelId { K_NODE_TAG = 0, K_FACE_TAG, K_CELL_TAG, K_RECON, K_FACE_SWEEP, K_FLUX, K_UPDATE, K_FLUX_PREP, K_FLUX_SUM, K_FLUX_OVER, K_FLUX_GEN, K_FLUX_DEEP, K_FLUX_GEN_UNITS, K_FLUX_GEN_SUM, K_FLUX_GEN_UDEEP, K_LSFIR_FIT, K_PLIC, K_ISO, K_COUNT };
// Optional per-kernel event bracketing: before(k)/after(k) are called around kernel k's launch.
struct Prof {
  virtual ~Prof() {}
  virtual void before(int k) = 0;
  virtual void after(int k) = 0;
};
// Launch shapes (none changes any result): block size of the vertex / face /
// cell sweeps, block size of the reconstruction, grid of the staging kernel
// (one wavefront per block), blocks per pair-buffer region of the pair and unit
// kernels, lanes per pair of the general-cell filter, the most faces and
// (face, cell, flux tet) pairs staged per step (0: as many as the workspace
// holds; what does not fit goes to the overflow and deferred kernels, which
// give the same values), lanes per face of the staging kernel, and units
// ranked together per thread of the general-cell unit kernel.
struct LaunchCfg {
  int sweep_threads = 256;
  int recon_threads = 128;
  int prep_blocks = 16384;
  int pair_blocks_per_region = 16;
  int filter_lanes = 0;  // 0: the general-cell filter by runs
  int staged_faces = 0;
  int staged_pairs = 0;
  int prep_lanes = 64;
  int units_rank = 4;  // general-cell units ranked together per thread of the unit kernel (4 or 8)
};
hipError_t launch_zero(int* p, int n, hipStream_t s);
hipError_t launch_geometry(const DevMesh& M, hipStream_t s);
// LSFIR and isosurface thresholds (host-computed, so every side takes the
// same bits): the cosines of 45 degrees (valid neighbours), of the stopping
// tolerance, of 1.2 rad and of 30/I degrees for each outer pass
// I = 1..kMaxLsfirOuter.
struct LsfirConsts {
  double cos_valid, cos_stop;
  double cos_iso;  // cos 1.2 rad: ELCIR / CLCIR keep their normal within this of the reference
  double cos_turn[kMaxLsfirOuter + 1];
};
hipError_t launch_reconstruct(const DevMesh& M, double* F, const LaunchCfg& L, hipStream_t s, Prof* prof = nullptr,
                              const LsfirConsts* lsfir = nullptr);
// reset: clear the step's counters first (not needed right after
// launch_reconstruct, whose first kernel clears them)
hipError_t launch_advect(const DevMesh& M, const double* uf, const double* uv, double dt, const double* Fin,
                         double* Fout, const LaunchCfg& L, hipStream_t s, Prof* prof = nullptr, bool reset = true);
hipError_t launch_face_tags(const DevMesh& M, hipStream_t s);
hipError_t launch_tri_cache(const DevMesh& M, hipStream_t s);
hipError_t launch_init(const DevMesh& M, int kind, const double* p, int ndiv, double* F, hipStream_t s);
// Device address and size of the library's static staging array on the
// current device (resolved on the first call on each device).
hipError_t static_scratch(void** ptr, size_t* bytes);
}  // namespace gvof
