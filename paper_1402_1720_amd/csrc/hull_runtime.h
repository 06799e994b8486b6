// Internal interface between the per-scan calls and the batch / server
// runtime: one job = one per-scan call with device pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "hullmi.h"

namespace hullmi {

// HULL_OK when the job's per-scan call would accept its arguments.
int job_check(const hullmi_job &j);
// Workspace bytes the job's call needs.
size_t job_ws_bytes(const hullmi_job &j);
// Enqueues the job's call on s; walk_blocks > 0 caps the persistent walk grid.
int job_run(const hullmi_job &j, void *ws, size_t ws_bytes, hipStream_t s, int walk_blocks);
// Device bytes of a request held entirely by the library (hull_footprint_bytes).
size_t footprint_bytes(int op, const hullmi_grid *grid, int64_t n, const hullmi_fbp_params *fbp);

}  // namespace hullmi
