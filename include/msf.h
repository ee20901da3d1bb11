/*
 * msf.h -- C ABI of the MI355X (gfx950) minimum spanning forest library.
 *
 * The library computes the minimum spanning forest of an undirected weighted
 * graph with the algebraic Awerbuch-Shiloach method of Baer, Kanakagiri and
 * Solomonik, "Parallel Minimum Spanning Forest Computation using Sparse
 * Matrix Kernels" (arXiv 2110.04865): rounds of a multilinear kernel over
 * the adjacency matrix and the parent vector (section 3.1), projection onto
 * supervertices, star hooking with tie breaking (Algorithm 2), and complete
 * shortcutting of the parent forest (section 4.2).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an msf_status and never aborts.  On any error the
 *    caller's output arrays and scalars are left untouched, and
 *    msf_last_error() returns a message for the calling thread.
 *  - Vertices are 0-based int32 ids.  Edge e of m is the pair
 *    (edges[2e], edges[2e+1]) with weight weights[e]; its id is e.
 *  - Edge order: key(e) = (wkey(w_e), e), compared lexicographically, where
 *    wkey is the weight for MSF_W_U32 and an order-preserving unsigned map of
 *    the bits for MSF_W_F32 (-0.0 equals +0.0).  The paper assumes distinct
 *    weights (section 2); breaking ties by edge id makes the forest unique,
 *    so results are deterministic and independent of every tuning choice.
 *  - Self-loops are accepted and never enter the forest; parallel edges are
 *    accepted and the one with the smaller key wins.
 *  - Ownership: the caller owns every array it passes; the library owns only
 *    the opaque handles it returns, released by the matching *_destroy.
 *    Inputs are read during the call (or copied, for graphs and server
 *    requests); nothing aliases a caller array after return.
 *  - msf_mem selects where caller arrays live.  MSF_MEM_HOST: host memory,
 *    the call is synchronous.  MSF_MEM_DEVICE: device memory on the context's
 *    device; work is ordered on the context's stream, and the call returns
 *    after its host scalar outputs are known (which synchronises the stream).
 *  - Errors: MSF_EINVAL for bad arguments (n < 0, m < 0, m > MSF_MAX_EDGES, an
 *    endpoint outside [0, n), a NaN weight, NULL with a nonzero size, a
 *    parent vector that is not a rooted forest), MSF_ENOMEM when device or
 *    host memory cannot be allocated, MSF_EDEVICE for a HIP runtime failure,
 *    MSF_EBUDGET when a server request cannot fit its memory budget,
 *    MSF_ENOTFOUND for an unknown server ticket.
 */
#ifndef MSF_H
#define MSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSF_OK = 0,
    MSF_EINVAL = 1,
    MSF_ENOMEM = 2,
    MSF_EDEVICE = 3,
    MSF_EBUDGET = 4,
    MSF_ENOTFOUND = 5
} msf_status;

/*
 * Largest edge count per graph (per batch, in total): 2^31 - 2048.  Edge ids
 * must stay below the 32-bit empty-key sentinel, and the adjacency stores
 * both directions (2m entries) with 32-bit positions plus one 1024-entry
 * sweep chunk of padding.
 */
#define MSF_MAX_EDGES 2147481600LL

typedef enum { MSF_W_U32 = 0, MSF_W_F32 = 1 } msf_wtype;
typedef enum { MSF_MEM_HOST = 0, MSF_MEM_DEVICE = 1 } msf_mem;

/*
 * Forest weight (Algorithm 2 returns the sum of the weights of the edges
 * that hook).  u64: exact sum for MSF_W_U32 weights, 0 for MSF_W_F32.
 * f64: the exact real sum of the forest's weights rounded once to the
 * nearest double (ties to even), so it does not depend on summation order.
 */
typedef struct {
    uint64_t u64;
    double f64;
} msf_total;

/* Per-solve statistics of the last msf_solve / msf_solve_batched on a ctx. */
typedef struct {
    int32_t rounds;          /* multilinear sweeps executed                  */
    int32_t hook_rounds;     /* rounds in which at least one root hooked     */
    int32_t max_chase;       /* longest pointer chase of any shortcut        */
    int32_t filtered;        /* number of filtering compactions done         */
    int64_t hooks[64];       /* hooks kept after tie breaking, per round     */
    int64_t active_nnz[64];  /* stored directions swept, per round           */
    double build_ms;         /* adjacency build time (device events)         */
    double rounds_ms;        /* round loop time (device events)              */
    double sweep_ms[64];     /* multilinear sweep kernel time, per round     */
    double sweep_bytes[64];  /* algorithmic bytes of that sweep: 12 per
                                stored entry (column + key), 8 per row with
                                entries (row pointer + p of the row), 8 per
                                live root (its minimum slot)                 */
    int32_t head_sweeps;     /* rounds swept over key-sorted runs (heads
                                only; their sweep_bytes are 0)               */
    int32_t path;            /* msf_solve: 0 rounds of device-wide launches,
                                one host round trip per round; 1 one
                                workgroup solved the whole graph in LDS
                                (small graphs; rounds and hooks are set,
                                rounds_ms is its kernel time); 2 rounds
                                driven on the device, several per host
                                round trip (full sweep, no filtering); 3
                                the same, replayed from a captured HIP
                                graph                                        */
    int64_t runs;            /* key-sorted runs of the adjacency (0: none)   */
    /* Device time (events) and algorithmic bytes of one-launch passes, 0
       when not run.  Index 0: placement of the two-level build (per stored
       entry its level-2 record read, column and key written; per vertex its
       row pointer, + round 1's minimum when the build keeps it).  1: run
       sort of the head sweep (24 per stored entry: column and key read and
       written; 16 per run: start read, head written; 4 per 64-entry
       chunk).  2: level-2 partition (per stored entry its level-1 record
       read, level-2 record and 2-byte row written).  3: level-1 partition
       (12 per edge read: endpoints and weight; per stored entry its level-1
       record and 1-byte fine bucket written). */
    double pass_ms[4];
    double pass_bytes[4];
    /* msf_solve_batched only: the persistent launch's candidate
       configuration (msf_batch_configs index; -1 when none ran), its
       workgroups, the graphs it solved, the graphs solved one by one
       instead (too large for one workgroup), and its device time. */
    int32_t batch_config;
    int32_t batch_grid;
    int64_t batch_graphs;
    int64_t batch_large;
    double batch_ms;
    /* msf_solve on the device-wide path with MSF_CHECK_ROUNDS=1 only (0
       otherwise): vertices that are roots (p[v] == v) at the start of each
       round.  In that mode every round is checked: every tree is a star
       after the shortcut, and the roots drop by exactly the kept hooks
       (MSF_EDEVICE otherwise). */
    int64_t roots[64];
    /* msf_solve with the two-level build: the adjacency build alone (device
       events from the solve's start to the end of the placement; build_ms
       also holds the head sweep's run set-up and the host step between
       them); 0 with the other builds. */
    double adjacency_ms;
} msf_stats;

typedef struct msf_ctx msf_ctx;
typedef struct msf_graph msf_graph;
typedef struct msf_server msf_server;

/*
 * Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (for example torch.cuda.current_stream().cuda_stream) or NULL for the
 * device's null stream.  The context caches device workspace between calls;
 * calls on one context must not overlap in time.
 */
msf_status msf_ctx_create(int device, void *hip_stream, msf_ctx **out);
/* Releases the context.  Every graph and server made on it must be
 * destroyed first (they use its stream and workspace). */
void msf_ctx_destroy(msf_ctx *ctx);

/* Thread-local message describing the last error ("" if none). */
const char *msf_last_error(void);

/* Library version string. */
const char *msf_version(void);

/*
 * Minimum spanning forest (section 2 problem statement; Algorithm 2 with
 * complete shortcutting, section 4.2).
 *   n, m            vertex and edge counts (n >= 0, 0 <= m <= MSF_MAX_EDGES)
 *   edges           int32[2m] endpoint pairs        (host or device per mem)
 *   weights         uint32[m] or float32[m] per wtype (host or device)
 *   forest_ids      int32[>= max(n-1,0)] out: forest edge ids, ascending
 *                   (host or device per mem)
 *   forest_count    host out: number of forest edges (= n - #components)
 *   total           host out (nullable): forest weight
 */
msf_status msf_solve(msf_ctx *ctx, int32_t n, int64_t m, const int32_t *edges,
                     const void *weights, msf_wtype wtype, msf_mem mem, int32_t *forest_ids,
                     int64_t *forest_count, msf_total *total);

/* Statistics of the last solve on ctx (host out). */
msf_status msf_get_stats(const msf_ctx *ctx, msf_stats *out);

/*
 * Build and keep the device adjacency structure of a graph: the symmetric
 * adjacency matrix A of section 2 (a_ij = w(i,j), both directions stored,
 * each carrying its edge's key).  Arguments as for msf_solve; the arrays are
 * copied.  *out receives a handle released by msf_graph_destroy.  The
 * vertices are stored in order of decreasing degree class (bit length of
 * the degree, ties by id), so the parents the multilinear kernel gathers
 * most share cache lines; every call on the graph takes and returns vectors
 * in the caller's vertex order (environment MSF_GRAPH_ORDER=0 keeps the
 * caller's order inside as well).
 */
msf_status msf_graph_create(msf_ctx *ctx, int32_t n, int64_t m, const int32_t *edges,
                            const void *weights, msf_wtype wtype, msf_mem mem,
                            msf_graph **out);
void msf_graph_destroy(msf_graph *g);

/*
 * The multilinear kernel of section 3.1 fused with the projection of
 * Algorithm 2 (its multilinear kernel and projection), for any parent vector p:
 *   r[k] = min { key(e) : stored direction i->j of edge e, p[i] == k,
 *                         p[i] != p[j] },  UINT64_MAX where the set is empty,
 * with key(e) = (uint64_t)wkey(w_e) << 32 | e.
 *   p   device uint32[n], every entry < n (MSF_EINVAL otherwise)
 *   r   device uint64[n] out
 * Ordered on the context's stream; returns without synchronising.
 * msf_get_stats afterwards describes this call as one round: sweep_ms[0] is
 * the sweep kernel's device time (events on the context's stream around that
 * one launch; msf_get_stats waits for them) and sweep_bytes[0] its streamed
 * bytes (12 per stored entry, 8 per row with entries, 4; the written slots
 * of r are not counted).  A graph stores its vertices by decreasing degree
 * class (msf_graph_create); p is first gathered into that order by a kernel
 * of its own, timed in pass_ms[0] with pass_bytes[0] = 12 per vertex.
 */
msf_status msf_multilinear(msf_ctx *ctx, const msf_graph *g, const uint32_t *p, uint64_t *r);

/*
 * One owner's share of the multilinear kernel when the rows of A are split
 * among several devices that each hold the whole parent vector (section 5
 * distributes A; here one device computes the share of a contiguous block
 * of stored rows): r as for msf_multilinear, but over the stored directions
 * whose row is one of the stored rows row_lo .. row_hi - 1 only.  The
 * shares of a partition of the rows combine by element-wise minimum into
 * msf_multilinear's r.
 *   row_lo, row_hi  0 <= row_lo <= row_hi <= n, positions in the graph's
 *                   stored vertex order (msf_graph_order); MSF_EINVAL
 *                   outside that range, or for a graph stored as several
 *                   column slices (MSF_SLICES)
 *   p, r            as for msf_multilinear (r is written for all n vertices)
 * Ordered on the context's stream; synchronises once before the sweep (to
 * read the range's entry bounds).  Statistics as for msf_multilinear, with
 * sweep_bytes[0] counting the range's entries and rows.
 */
msf_status msf_multilinear_rows(msf_ctx *ctx, const msf_graph *g, const uint32_t *p, uint64_t *r,
                                int32_t row_lo, int32_t row_hi);

/*
 * The graph's stored vertex order: order[k] = the caller's id of the vertex
 * stored as row k (the identity for a graph kept in the caller's order).
 *   order  device uint32[n] out
 * Returns after synchronising.
 */
msf_status msf_graph_order(msf_ctx *ctx, const msf_graph *g, uint32_t *order);

/*
 * The same r by the pairwise formulation of section 4.1, for comparing the
 * two: a first pass stores the pair (a_ij, p_j) of every stored entry (the
 * column parent p_j beside the entry's key: nnz extra writes of 4 bytes), a
 * second computes f(p_i, (a_ij, p_j)) and the projection from those pairs.
 * Arguments, result and errors as for msf_multilinear.  The pair array lives
 * in the context's workspace (grown, never shrunk: 4 bytes per slot of the
 * graph's padded column array, about 8 bytes per edge).
 */
msf_status msf_multilinear_pairwise(msf_ctx *ctx, const msf_graph *g, const uint32_t *p,
                                    uint64_t *r);

/*
 * Complete shortcutting (section 4.2): p[i] <- the root of i's tree in the
 * parent forest p (p[root] == root).  p is device uint32[n], in/out.
 * sub_iters (host, nullable) receives the number of pointer-jumping passes.
 * MSF_EINVAL, with p untouched, if some p[i] >= n or p is not a rooted forest
 * (it has a cycle longer than one).
 */
msf_status msf_shortcut(msf_ctx *ctx, int32_t n, uint32_t *p, int32_t *sub_iters);

/*
 * Complete shortcutting by a chosen strategy, for the shortcut study of
 * section 7.1 in single-device form.  A pass (a sub-iteration of section 7.1)
 * moves each taking part vertex to its grandparent:
 *   MSF_SHORTCUT_FRONTIER  only vertices whose parent is not yet a root take
 *                          part (the counterpart of CSP, which shortcuts only
 *                          the data it gathered once); msf_shortcut does this;
 *   MSF_SHORTCUT_FULL      every vertex takes part in every pass (the
 *                          baseline: each vertex queries its parent in every
 *                          sub-iteration);
 *   MSF_SHORTCUT_SWITCH    full passes until at most switch_fraction * n
 *                          vertices are unfinished, then the frontier (OS,
 *                          with its threshold taken per pass instead of per
 *                          iteration).
 * switch_fraction (in [0, 1]) is read by MSF_SHORTCUT_SWITCH only.  Result,
 * sub_iters (passes of either kind) and errors as for msf_shortcut;
 * MSF_EINVAL for an unknown strategy or a fraction outside [0, 1].
 */
enum { MSF_SHORTCUT_FRONTIER = 0, MSF_SHORTCUT_FULL = 1, MSF_SHORTCUT_SWITCH = 2 };
msf_status msf_shortcut_strategy(msf_ctx *ctx, int32_t n, uint32_t *p, int32_t strategy,
                                 double switch_fraction, int32_t *sub_iters);

/*
 * Connected components by the same rounds, in the connectivity variant of
 * the Awerbuch-Shiloach algorithm (section 2.4): each star root hooks along
 * an edge leaving its star (here the minimum-key one, from the multilinear
 * kernel), the smaller of two roots that hooked onto each other stays root,
 * and complete shortcutting over the hooked roots makes every tree a star
 * again.  On a graph where msf_solve takes the head sweep (one column slice,
 * at least 2^20 stored entries and 16 per vertex, or MSF_HEADS=2) the rounds
 * are msf_solve's, over a copy of the graph's entries sorted by (row, key)
 * in 64-entry chunks; otherwise they run on the device four at a time, with
 * the host reading the termination flag between groups.  The graph is only
 * read.
 *   labels  device uint32[n] out: labels[i] == labels[j] iff i and j are
 *           connected; each label is a vertex of its component (the root
 *           its tree ended at, not necessarily the smallest id)
 *   rounds  (host, nullable) receives the number of hooking rounds
 * Ordered on the context's stream; returns after synchronising.  Uses the
 * context's workspace (as msf_solve on the same graph, or 24 bytes per
 * vertex and 1 per edge); msf_get_stats afterwards describes the rounds.
 */
msf_status msf_components(msf_ctx *ctx, const msf_graph *g, uint32_t *labels, int32_t *rounds);

/*
 * The minimum spanning forest by the original Awerbuch-Shiloach rounds
 * (section 2.3, Algorithm 1), for comparison with complete shortcutting:
 * each round flags the stars (star check), lets every star root hook along
 * its star's minimum-key outgoing edge onto the parent of the outside
 * endpoint (the smaller of two roots that hooked onto each other stays
 * root), then shortcuts every vertex by one step.  Stops after a round with
 * no hook and no change.
 *   in_forest  device uint8[m] out: 1 for the edges of the forest (the same
 *              forest as msf_solve), 0 otherwise
 *   rounds     (host, nullable) receives the number of rounds
 * Ordered on the context's stream; returns after synchronising.  Uses the
 * context's workspace (24 bytes per vertex).
 */
msf_status msf_solve_starcheck(msf_ctx *ctx, const msf_graph *g, uint8_t *in_forest,
                               int32_t *rounds);

/*
 * Minimum spanning forests of G independent graphs in one batched solve.
 * Graph g has vtx_off[g+1]-vtx_off[g] vertices and edge_off[g+1]-edge_off[g]
 * edges stored from edges[2*edge_off[g]] (local vertex ids) and
 * weights[edge_off[g]].  vtx_off/edge_off are host int64[G+1] starting at 0
 * and non-decreasing.  Outputs (per mem): forest_ids int32[vtx_off[G]]
 * receives graph g's forest (local edge ids, ascending) from index
 * vtx_off[g]; counts int64[G] (host) and totals msf_total[G] (host,
 * nullable).  Each graph's result equals msf_solve on that graph alone.
 */
/*
 * Launch configurations the batched solve chooses from (its tuner times
 * each on a sample of a batch and caches the fastest per batch shape; the
 * environment variable MSF_BATCH_CONFIG=<index> forces one).  Writes up to
 * cap entries: threads per workgroup, edges each thread loads per step of a
 * sweep, and dynamic LDS bytes per workgroup (graphs whose state fits it
 * are solved in LDS).  Returns the number of candidates; arrays may be NULL
 * to query the count.  Every candidate gives bit-identical results.
 */
int msf_batch_configs(int32_t *nt, int32_t *ept, int32_t *lds_bytes, int32_t cap);

msf_status msf_solve_batched(msf_ctx *ctx, int32_t G, const int64_t *vtx_off,
                             const int64_t *edge_off, const int32_t *edges, const void *weights,
                             msf_wtype wtype, msf_mem mem, int32_t *forest_ids, int64_t *counts,
                             msf_total *totals);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * batched solve with every array in device memory and every scratch buffer
 * in a fixed array of MSF_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends.  The call allocates nothing.
 *   vtx_off, edge_off  device int64[G+1], starting at 0, non-decreasing
 *   edges, weights     device, as for msf_solve_batched (local vertex ids)
 *   forest_ids         device int32[vtx_off[G]] out: graph g's forest
 *                      (local edge ids, ascending) from index vtx_off[g]
 *   counts             device int64[G] out
 *   totals             device msf_total[G] out
 * Every graph must have at most 2^20 vertices and 2^22 edges, and its
 * working set (32 bytes per edge + 20 per vertex + flags) must fit the
 * array (MSF_EINVAL otherwise); the array holds as many graphs in flight as
 * fit (fewer for larger graphs).  Offsets, endpoints and weights are checked
 * in a first pass, so on any error nothing is written.  The call returns
 * once that check is done (it synchronises the context's stream); the solve
 * itself stays ordered on the stream.  Every call on one GPU uses the same
 * array: calls that overlap in time on a GPU race.  Each graph's result
 * equals msf_solve_batched's (and msf_solve's on that graph alone).
 */
#define MSF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
msf_status msf_solve_batched_noalloc(msf_ctx *ctx, int32_t G, const int64_t *vtx_off,
                                     const int64_t *edge_off, const int32_t *edges,
                                     const void *weights, msf_wtype wtype, int32_t *forest_ids,
                                     int64_t *counts, msf_total *totals);

/*
 * Serving: a request loop with continuous batching.  Requests are admitted
 * while their device footprint fits mem_budget_bytes; admitted requests keep
 * their adjacency, parent and edge state resident on the device and advance
 * together, one batched round per step, on a worker thread; finished
 * requests retire and free their memory for waiting ones.
 *   msf_server_submit copies the host arrays and returns a ticket; it fails
 *   with MSF_EBUDGET if the request alone can never fit the budget.
 *   msf_server_poll sets *done to 1 once the result is ready.
 *   msf_server_result waits for the result, writes it (host arrays, as for
 *   msf_solve with MSF_MEM_HOST) and releases the ticket.
 *   msf_server_latency gives (host, seconds) submit-to-ready latency of a
 *   finished ticket.
 */
msf_status msf_server_create(msf_ctx *ctx, size_t mem_budget_bytes, msf_server **out);
void msf_server_destroy(msf_server *s);
msf_status msf_server_submit(msf_server *s, int32_t n, int64_t m, const int32_t *edges,
                             const void *weights, msf_wtype wtype, uint64_t *ticket);
msf_status msf_server_poll(msf_server *s, uint64_t ticket, int *done);
msf_status msf_server_latency(msf_server *s, uint64_t ticket, double *seconds);
msf_status msf_server_result(msf_server *s, uint64_t ticket, int32_t *forest_ids,
                             int64_t *forest_count, msf_total *total);

/* Device bytes a request of this size occupies while resident (an upper
   bound over every path a solve takes: builds, full or head sweep). */
size_t msf_request_footprint(int32_t n, int64_t m);

#ifdef __cplusplus
}
#endif

#endif /* MSF_H */
