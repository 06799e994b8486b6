// Internal interface between the per-scan calls and the batch / server
// runtime: one job = one per-scan call with device pointers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "hullmi.h"

namespace hullmi {

// Event pairs recorded around kernel launches (a measurement aid:
// hull_count_profile, hull_fbp_profile), one pair per launch, tagged with the
// kernel's hull_prof_kernel id. Events are created as launches are made and
// destroyed with the object.
struct KernelProf {
    struct Mark {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    bool failed = false;
    void begin(int k, hipStream_t s)
    {
        Mark m{k, nullptr, nullptr};
        if (hipEventCreate(&m.a) != hipSuccess || hipEventCreate(&m.b) != hipSuccess ||
            hipEventRecord(m.a, s) != hipSuccess) {
            failed = true;
            if (m.a) (void)hipEventDestroy(m.a);
            if (m.b) (void)hipEventDestroy(m.b);
            return;
        }
        marks.push_back(m);
    }
    void end(hipStream_t s)
    {
        if (!marks.empty() && hipEventRecord(marks.back().b, s) != hipSuccess) failed = true;
    }
    ~KernelProf()
    {
        for (const Mark &m : marks) {
            (void)hipEventDestroy(m.a);
            (void)hipEventDestroy(m.b);
        }
    }
};

// Launch choices of the counting pass; 0 keeps the library's default.
struct CountOpts {
    int walk_blocks = 0;        // cap on the workgroups of the persistent walk
    int ranges_per_group = 0;   // equal-work ranges per walk workgroup
    int length_classes = 0;     // line-length classes per slice (at most the default)
    int run_stride = 0;         // block stride of the item runs
    // per-scan calls: a pass of several internal batches splits the workspace
    // in two and alternates batches between the caller's stream and a second
    // one (sequentially, in the same batches, when prof is set)
    bool two_streams = false;
    KernelProf *prof = nullptr;  // event pairs around every launch
};

// HULL_OK when the job's per-scan call would accept its arguments.
int job_check(const hullmi_job &j);
// Workspace bytes the job's call needs.
size_t job_ws_bytes(const hullmi_job &j);
// Enqueues the job's call on s with the counting pass's launch choices o.
int job_run(const hullmi_job &j, void *ws, size_t ws_bytes, hipStream_t s, const CountOpts &o);
// Device bytes of a request held entirely by the library (hull_footprint_bytes).
size_t footprint_bytes(int op, const hullmi_grid *grid, int64_t n, const hullmi_fbp_params *fbp);

// Pieces of the per-scan calls for a session that keeps counts resident.
bool params_ok(const hullmi_params *p);
bool grid_valid(const hullmi_grid *g);
bool hist_valid(const hullmi_histories *h);
size_t counting_ws_bytes(const hullmi_grid *g, int64_t n);   // counting, up to n histories a call
size_t rules_ws_bytes(const hullmi_grid *g);                 // masks from counts
// Adds the counts of h to N and M (and its counters to stats), with a counting
// workspace of ws_bytes.
int counts_accumulate(const hullmi_histories *h, const hullmi_grid *g, const hullmi_params *p,
                      int32_t *N, int32_t *M, hullmi_stats *stats, void *ws, size_t ws_bytes,
                      hipStream_t s);
// The SC, MSC and SM masks of counts N and M (each mask may be null).
int masks_from_counts(const hullmi_grid *g, const hullmi_params *p, const int32_t *N,
                      const int32_t *M, uint8_t *sc, uint8_t *msc, uint8_t *sm, void *ws,
                      hipStream_t s);
void zero_counts(int32_t *N, int32_t *M, hullmi_stats *stats, int64_t V, hipStream_t s);

}  // namespace hullmi
