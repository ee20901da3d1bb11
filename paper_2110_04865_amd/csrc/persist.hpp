// Persistent batched solve (kernels_persist.hip) and its tuning
// (tune.hip): shared declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>

#include "msf_internal.hpp"

namespace msf {

// Arguments of one persistent launch.  Graph g has vtx_off[g+1]-vtx_off[g]
// vertices and edge_off[g+1]-edge_off[g] edges (local endpoint ids, weight
// bits); order lists the graphs to solve (largest first; null: every graph
// in index order), queue is the shared cursor into it.  Each workgroup owns slot_bytes of scratch: two
// live-edge buffers of m_cap entries (16 bytes each), then the state of a
// graph too large for LDS (persist_state_bytes(n_cap, m_cap)).
struct PersistArgs {
    int32_t G = 0;
    const uint32_t *order = nullptr;
    uint32_t *queue = nullptr;
    const int64_t *vtx_off = nullptr;
    const int64_t *edge_off = nullptr;
    const int32_t *edges = nullptr;
    const uint32_t *w = nullptr;
    int32_t *out = nullptr;
    int64_t *counts = nullptr;
    uint64_t *tot_u64 = nullptr;
    double *tot_f64 = nullptr;
    uint8_t *scratch = nullptr;
    size_t slot_bytes = 0;
    uint32_t m_cap = 0;
    uint32_t lds_bytes = 0;
    uint32_t *err = nullptr;
    // nullable: kept hooks of rounds 0..63 and, at [64], the rounds run
    // (for a launch that solves one graph)
    uint32_t *round_hooks = nullptr;
    // graph g's totals go to tot_u64[g * tot_stride], tot_f64[g * tot_stride]
    // (2 when they are the fields of an msf_total array)
    uint32_t tot_stride = 1;
};

// A launch configuration: threads per workgroup, edges each thread loads per
// step of a sweep, dynamic LDS per workgroup (graphs whose state fits it
// keep their state in LDS; it also sets how many workgroups share a CU).
struct PersistCfg {
    int nt;
    int ept;
    uint32_t lds;
};

// Graphs above these sizes are not solved by the persistent kernel.
constexpr uint32_t PERSIST_MAX_N = 1u << 20;
constexpr uint32_t PERSIST_MAX_M = 1u << 22;
// Dynamic LDS of the one-workgroup solve of a small graph (msf_solve).
constexpr uint32_t SMALL_LDS = 150u << 10;

__host__ __device__ inline size_t persist_state_bytes(uint32_t n, uint32_t m)
{
    return 20 * (size_t)n + 4 * (((size_t)m + 31) / 32);
}

__host__ inline size_t persist_slot_bytes(uint32_t n_cap, uint32_t m_cap)
{
    const size_t b = 2 * 16 * (size_t)m_cap + persist_state_bytes(n_cap, m_cap);
    return (b + 255) & ~(size_t)255;
}

// The candidate configurations the tuner times (count in *count).
const PersistCfg *persist_candidates(int *count);

// Zero the queue and error word, then launch `grid` workgroups.
hipError_t launch_persist(hipStream_t s, const PersistArgs &A, const PersistCfg &cfg, int wt,
                          unsigned grid);

// Offsets {0, n}, {0, m} and order {0} of a one-graph launch (a kernel).
void launch_small_setup(hipStream_t s, int64_t *vo, int64_t *eo, uint32_t *order, int64_t n,
                        int64_t m);

// Whether msf_solve takes the one-workgroup path for this graph: at most
// c->small_m edges and state that fits the largest LDS allocation.
bool small_eligible(const Ctx *c, int32_t n, int64_t m);

// msf_solve of a small graph by one workgroup of the persistent kernel
// (every round in LDS, no host round trips); same outputs as solve_device.
msf_status solve_small(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                       msf_wtype wt, int32_t *d_ids, int64_t *count, msf_total *total);

// Workgroups of this configuration one compute unit holds at once (0 if the
// configuration cannot run).
int persist_blocks_per_cu(const PersistCfg &cfg, int wt);

// Whether the configuration's dynamic LDS fits this device.
bool persist_cfg_fits(int device, const PersistCfg &cfg);

// Shape of a batch, for the tuning cache key.
struct BatchShape {
    double mean_n = 0.0;    // mean vertices per graph
    double mean_deg = 0.0;  // mean stored entries (2 m) per vertex
};

// Runs candidate `cand` once on a sample of the batch; with ms non-null it
// also times the run (device events).
using PersistTuneRun = std::function<msf_status(int cand, float *ms)>;

// The candidate to use for a batch of this shape: MSF_BATCH_CONFIG if set,
// else the cached choice, else the fastest candidate on the sample (then
// cached).
msf_status persist_pick(Ctx *c, const BatchShape &shape, int wt, const PersistTuneRun &run,
                        int *chosen);

}  // namespace msf
