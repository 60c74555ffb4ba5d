// kernels.h -- launchers of the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace bdu {

// Every launcher takes a device array of `count` device pointers to
// HandleDev and a Gate (which handles take part in this pass).  The
// projection reads column gate.pass of the staged B and C.
hipError_t launch_project(HandleDev *const *hs, int count, int max_tiles, Gate gate, hipStream_t st);
hipError_t launch_spike(HandleDev *const *hs, int count, Gate gate, hipStream_t st);
// threads: the largest plan thread count (Plan::L) of the launch's handles;
// a handle with fewer chains than threads runs one chain per thread.
hipError_t launch_gen(HandleDev *const *hs, int count, int64_t lds_bytes, bool in_lds, int threads, Gate gate,
                      hipStream_t st);
hipError_t launch_apply(HandleDev *const *hs, int count, int max_panels, int k0, int nw, int rpl, Gate gate,
                        hipStream_t st);
// One-time kernel attributes; call before capturing launches in a graph.
hipError_t prepare_kernels();
hipError_t launch_fill_identity(double2 *p, int64_t count, hipStream_t st);
// flag[0] = 1 if any of p[0..count) is NaN or infinite (caller clears flag).
hipError_t launch_nonfinite(const double *p, int64_t count, int *flag, hipStream_t st);
bool tiling_supported(int k0, int nw, int rpl);
hipError_t launch_givens(const double *a, const double *b, int mode, double *c, double *s, double *r,
                         int64_t count, hipStream_t st);

}  // namespace bdu
