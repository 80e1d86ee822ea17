// Host-side launchers of the gVOF kernels (defined in gvof_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gvof_dev.h"

namespace gvof {
hipError_t launch_zero(int* p, int n, hipStream_t s);
hipError_t launch_geometry(const DevMesh& M, hipStream_t s);
hipError_t launch_reconstruct(const DevMesh& M, double* F, hipStream_t s);
hipError_t launch_advect(const DevMesh& M, const double* uf, const double* uv, double dt, const double* Fin,
                         double* Fout, hipStream_t s);
hipError_t launch_init(const DevMesh& M, int kind, const double* p, int ndiv, double* F, hipStream_t s);
}  // namespace gvof
