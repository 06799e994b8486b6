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

// Pieces of the per-scan calls for a session that keeps counts resident.
bool params_ok(const hullmi_params *p);
bool grid_valid(const hullmi_grid *g);
bool hist_valid(const hullmi_histories *h);
size_t counting_ws_bytes(const hullmi_grid *g, int64_t n);   // counting, up to n histories a call
size_t rules_ws_bytes(const hullmi_grid *g);                 // masks from counts
// Adds the counts of h to N and M (and its counters to stats).
int counts_accumulate(const hullmi_histories *h, const hullmi_grid *g, const hullmi_params *p,
                      int32_t *N, int32_t *M, hullmi_stats *stats, void *ws, hipStream_t s);
// The SC, MSC and SM masks of counts N and M (each mask may be null).
int masks_from_counts(const hullmi_grid *g, const hullmi_params *p, const int32_t *N,
                      const int32_t *M, uint8_t *sc, uint8_t *msc, uint8_t *sm, void *ws,
                      hipStream_t s);
void zero_counts(int32_t *N, int32_t *M, hullmi_stats *stats, int64_t V, hipStream_t s);

}  // namespace hullmi
