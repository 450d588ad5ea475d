// Host-side launchers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

namespace sdd {

hipError_t launch_camgen(const CamParams& p, hipStream_t st);
hipError_t launch_trace(const TraceParams& p, bool count, int grid_blocks, hipStream_t st);
int trace_blocks_per_cu(int n_cells);  // resident trace workgroups per CU for a grid of n_cells subdomains
hipError_t launch_shade(const ShadeParams& p, hipStream_t st);
hipError_t launch_route(const RouteParams& p, hipStream_t st);
hipError_t launch_spectral(const SpectralParams& p, hipStream_t st);
// radiance-cache training rows of the training paths of one batch segment
hipError_t launch_nrc_rows(const NrcRowParams& p, hipStream_t st);
hipError_t launch_resolve(int WH, int nl, int nlp, double inv_spp, const float* acc, const double* w,
                          const double* cmf, double* spectral, double* xyz, hipStream_t st);
hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st);
// dst[i] |= *src, i < n (stream-ordered; a kernel, so graph capture records no memset)
hipError_t launch_fold_flags(const int* src, int* const* dst, int n, hipStream_t st);
hipError_t launch_pane(int n, const float4* pc, const float* c, float2* out, hipStream_t st);
// q[i] = (glass index, wavelength index, signed cosine bits, 0)
hipError_t launch_glass(int n, const GlassTable& tab, const int4* q, float2* out, hipStream_t st);
hipError_t launch_philox(int n, const uint4* ctr, uint2 key, uint4* out, hipStream_t st);
hipError_t launch_debug_rays(int n, const float* o, const float* d, const GridParams& grid, float2* hit, float4* qa,
                             float4* qb, int2* qc, int* cnt, long long cap, hipStream_t st);

}  // namespace sdd
