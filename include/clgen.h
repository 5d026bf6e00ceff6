/*
 * clgen.h -- C ABI of the MI355X (gfx950) Chung-Lu edge generator.
 *
 * Problem (Alam & Khan, "Parallel Algorithms for Generating Random Networks
 * with Given Degree Sequences", Sec. 3): given n non-negative weights
 * w_0 >= w_1 >= ... >= w_{n-1} and S = sum_k w_k, produce a random graph in
 * which every pair {u,v} is an edge independently with probability
 * min(w_u w_v / S, 1).  The generator is Create-Edges(w, S, V) of Alg. 1
 * (geometric skipping): S and the source range V are explicit inputs.
 *
 * Conventions for every call:
 *   - pointers are device pointers unless the comment says "host";
 *   - `stream` is a hipStream_t (NULL = the null stream); work is enqueued on
 *     it; calls documented as "synchronises" wait for their own work;
 *   - the caller owns every buffer (weights, workspace, edges); the library
 *     never allocates device memory and keeps no state between calls (the
 *     one exception: the fixed per-GPU array of cl_sample_into_noalloc);
 *   - errors are returned as negative cl_status values, never thrown.
 *
 * Output of the generator: uint32 pairs (u, v) with u < v, sorted by (u, v),
 * node ids being positions in the sorted weight vector.  The edge list is a
 * pure function of (w, S, seed, range): it does not depend on the launch
 * schedule, the lane budget or the number of graphs in a batch.
 *
 * Sampling rule (the points Alg. 1 leaves open, fixed so that any conforming
 * implementation gives the same bits):
 *   - random words: Philox4x32-10 with counter (t, k, u, 0) and key
 *     (seed mod 2^32, seed >> 32); t counts the draws of segment k of source u;
 *   - uniforms r_skip = U53(x1:x0), r_acc = U53(x3:x2), U53(x) = (2(x>>12)+1) 2^-53;
 *   - p = min((w_u / S) w_v, 1); skip delta = floor(LN(r_skip) / LN1M(p)) with
 *     binary64 logs built from a fixed range reduction and an 11-term atanh
 *     series; the segment ends when the skip leaves it; keep v iff r_acc p < q;
 *   - sources whose expected edge count e_u (Eq. 1 on the quantised prefix
 *     q_v = floor(w_v 2^32 / w_0)) exceeds 256 are split into
 *     min(ceil(e_u / 256), n-u-1) segments of equal quantised mass.
 */
#ifndef CLGEN_H_
#define CLGEN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cl_status;

#define CL_OK               0
#define CL_ERR_INVALID_ARG (-1)  /* bad pointer/size/range, S <= 0, S < w_0, 0 < w_0 < 2^-960 */
#define CL_ERR_UNSORTED    (-2)  /* weights not non-increasing (Sec. 3 input condition) */
#define CL_ERR_NEGATIVE    (-3)  /* a negative weight */
#define CL_ERR_NONFINITE   (-4)  /* a NaN or infinite weight (or an infinite sum) */
#define CL_ERR_TOO_LARGE   (-5)  /* n >= 2^32 (node ids are uint32) */
#define CL_ERR_WORKSPACE   (-6)  /* workspace too small; the required size is reported */
#define CL_ERR_CAPACITY    (-7)  /* a size exceeded what the workspace was laid out for */
#define CL_ERR_DEVICE      (-8)  /* a HIP runtime error, or an internal check failed on the device */
#define CL_ERR_NOT_PLANNED (-9)  /* workspace does not hold a plan from cl_count */

/* One generation task: Create-Edges(w, S, [u_begin, u_end)) of Alg. 1. */
typedef struct cl_graph {
  const double* w;     /* device, n weights, non-increasing, finite, >= 0 */
  uint64_t n;          /* < 2^32 */
  double S;            /* > 0, >= w[0]; normally the exact sum (cl_weight_sum) */
  uint64_t seed;       /* Philox key */
  uint64_t u_begin;    /* source range, 0 <= u_begin <= u_end <= n */
  uint64_t u_end;
} cl_graph;

/* Schedule knobs.  They change the launch schedule only, never an output bit
 * of the generator (the expected-degree tile shape changes only the float32
 * summation order of cl_expected_degree[_backward]).  Zero fields take the
 * defaults. */
typedef struct cl_tuning {
  uint32_t lane_budget;    /* expected candidates per lane (Eq. 5 chunk size), default 192 */
  uint32_t blocks_per_cu;  /* persistent grid = compute units x this (256-thread blocks), default 3 */
  uint32_t slot_margin;    /* cl_sample slots: 0 = mu + 8 sqrt(mu) + 24 (default); 1 = no margin (tests
                              of the overflow replay: about half of the lanes overflow) */
  uint32_t partition;      /* work units: 0 = equal expected cost (Eq. 5 applied to lanes, default);
                              1 = equal numbers of sources (the naive consecutive partition Sec. 4
                              compares against; heavy sources then serialise their unit);
                              2 = round robin (Sec. 4's RRP applied to segments: unit i of L takes
                              segments i, i + L, i + 2L, ...).  A round-robin unit's edges are not
                              contiguous in (u, v) order, so 2 is accepted by cl_plan only (then
                              cl_degrees); cl_count and cl_sample return CL_ERR_INVALID_ARG.
                              Other values: CL_ERR_INVALID_ARG. */
  uint32_t tail_units;     /* with partition 0: 0 = graded (default): the last 1/8 of a graph's
                              cost is cut into units 4 times smaller than lane_budget, so that the
                              lanes still busy when the work runs out finish close together
                              (graphs of at least 4096 units; in a batch only the last task, since
                              the queue hands out the tasks' units in order); 1 = uniform units */
  uint32_t ed_rows;        /* expected-degree tiles: rows per thread, 1, 2 (default) or 4 */
  uint32_t ed_cols;        /* expected-degree tiles: columns per tile, 512, 1024 (default) or 2048;
                              other values of either: CL_ERR_INVALID_ARG.  The tile shape changes
                              only the float32 summation order inside a tile */
  uint32_t unit_order;     /* order in which the lanes take the work units: 0 = default (2 for a
                              single graph, 1 for a batch); 1 = index order; 2 = by the position of
                              each unit's first candidate in the quantised prefix of w (512 bands of
                              equal prefix mass; graded units in a second run after the others), so
                              that the lanes in flight gather from a narrow stretch of w at a time and
                              share its cache lines.  2 needs a single-graph plan (G > 1:
                              CL_ERR_INVALID_ARG) and adds 4 bytes per unit and a count matrix to the
                              workspace.  Other values: CL_ERR_INVALID_ARG */
} cl_tuning;

/* ---------------------------------------------------------------------------
 * S <- sum_k w_k (Alg. 1, first line; Sec. 4 forms it by a parallel sum).  Returns the
 * exactly rounded sum (the real sum rounded once to nearest-even), which does
 * not depend on the summation order.  Also validates w (sorted, >= 0, finite).
 * ws: device workspace of cl_weight_sum_workspace() bytes.  S_out: host.
 * Synchronises.
 * ------------------------------------------------------------------------- */
cl_status cl_weight_sum_workspace(uint64_t n, uint64_t* bytes_out /* host */);
cl_status cl_weight_sum(const double* w, uint64_t n, void* ws, uint64_t ws_bytes,
                        double* S_out /* host */, void* stream);

/* ---------------------------------------------------------------------------
 * E[m] = sum_{u<v} min(w_u w_v / S, 1) (Eq. 1 with the cap; m = sum_u e_u of
 * Sec. 4) and Var[m] = sum_{u<v} p (1 - p), p as used by the sampler.  Float64,
 * sorted closed form (capped candidates of u form a prefix of v > u).
 * Em_out, Var_out: host.  Synchronises.
 * ------------------------------------------------------------------------- */
cl_status cl_expected_edges_workspace(uint64_t n, uint64_t* bytes_out /* host */);
cl_status cl_expected_edges(const double* w, uint64_t n, double S, void* ws, uint64_t ws_bytes,
                            double* Em_out /* host */, double* Var_out /* host */, void* stream);

/* ---------------------------------------------------------------------------
 * Uniform consecutive partition (Sec. 4, Eq. 2, Eq. 5, Alg. 2): bounds
 * n_0 = 0 <= n_1 <= ... <= n_P = n with n_k = min{u : C_u >= k Z / P}, where
 * C_u is the cumulative cost of sources 0..u, c_u = e_u + 1 (Eq. 2) with e_u
 * from Eq. 6 on the quantised prefix, kept in units of 1/256 (c_u =
 * floor(256 e_u) + 256) so that C_u is an exact integer, and Z = C_{n-1}.
 * Partition i is [n_i, n_{i+1}); partitions may be empty.
 * bounds_out: host, P + 1 entries.  Synchronises.
 * ------------------------------------------------------------------------- */
cl_status cl_partition_workspace(uint64_t n, uint32_t P, uint64_t* bytes_out /* host */);
cl_status cl_partition(const double* w, uint64_t n, double S, uint32_t P, void* ws, uint64_t ws_bytes,
                       uint64_t* bounds_out /* host */, uint64_t* total_cost_out /* host, may be NULL */,
                       void* stream);

/* ---------------------------------------------------------------------------
 * Generation, count pass (Alg. 1 run once to count).  Plans G independent
 * tasks in one workspace: validation, the quantised prefix, per-source costs
 * (Eq. 1-2) and segments, the lane plan (Eq. 5 applied to lanes), then counts
 * the edges of every lane and forms their output offsets.
 * m_out: host, G entries (edges per task).  ws_required (host, may be NULL)
 * receives the bytes the workspace needs; when ws_bytes is smaller the call
 * returns CL_ERR_WORKSPACE without generating (call again with a larger ws).
 * cl_workspace_size gives the size of the part known before the data is seen
 * (fixed_bytes) and an estimate of the whole (estimate_bytes) for cl_count
 * (one_pass = 0) or cl_sample (one_pass = 1).
 * Synchronises twice (sizes, counts).
 * ------------------------------------------------------------------------- */
cl_status cl_workspace_size(const cl_graph* g /* host, G entries */, uint32_t G, const cl_tuning* t,
                            uint32_t one_pass, uint64_t* fixed_bytes /* host */,
                            uint64_t* estimate_bytes /* host */);
cl_status cl_count(const cl_graph* g /* host, G entries */, uint32_t G, const cl_tuning* t,
                   void* ws, uint64_t ws_bytes, uint64_t* m_out /* host */,
                   uint64_t* ws_required /* host, may be NULL */, void* stream);

/* ---------------------------------------------------------------------------
 * Generation in one pass: the same plan as cl_count, then every lane runs
 * Alg. 1 once, counting its edges and writing them into its own slot of the
 * workspace as 32-bit words (v per edge, a mark and u where the source
 * changes; capacity from the lane's plan cost mu: mu + 8 sqrt(mu) + 24 edge
 * words, a Chernoff margin after Sec. 4, Theorem 2, plus two words per
 * segment; a lane above it is replayed by cl_generate).  m_out as for
 * cl_count.  cl_generate then expands the slots into the output instead of
 * replaying the lanes.  The workspace is larger than for cl_count by about
 * 1.5 x 4 bytes per expected edge.  Synchronises twice.
 * ------------------------------------------------------------------------- */
cl_status cl_sample(const cl_graph* g /* host, G entries */, uint32_t G, const cl_tuning* t,
                    void* ws, uint64_t ws_bytes, uint64_t* m_out /* host */,
                    uint64_t* ws_required /* host, may be NULL */, void* stream);

/* ---------------------------------------------------------------------------
 * cl_sample followed by cl_generate(ws, t, edges, 0, cap, graph_offsets)
 * without returning to the host in between: for callers that already hold
 * an output buffer (e.g. from an earlier run of the same shape).  The plan's
 * second half, the one pass, the expansion into edges and graph_offsets are
 * queued together; like cl_sample the call synchronises twice (sizes after
 * the plan's first half, counts at the end), with no host round trip between
 * the one pass and the expansion.  Returns
 * CL_ERR_CAPACITY when the total m exceeds cap: m_out is set, edges holds the
 * first cap edges and the plan stays valid for cl_generate with a larger
 * buffer.  Other arguments and errors as for cl_sample and cl_generate.
 * ------------------------------------------------------------------------- */
cl_status cl_sample_into(const cl_graph* g /* host, G entries */, uint32_t G, const cl_tuning* t,
                         void* ws, uint64_t ws_bytes, uint32_t* edges, uint64_t cap,
                         uint64_t* graph_offsets, uint64_t* m_out /* host */,
                         uint64_t* ws_required /* host, may be NULL */, void* stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc; code that replays captured work can
 * capture a counted plan with cl_batch_capture instead, since this call
 * synchronises like cl_sample_into and so cannot itself be captured):
 * cl_sample_into with the workspace taken from a fixed array of
 * CL_NOALLOC_SCRATCH_BYTES in device memory that the library holds, one
 * copy per GPU, from the loading of the library until the process ends.
 * The caller passes only inputs and outputs (g, edges, graph_offsets); the
 * call allocates no device memory (no hipMalloc / hipFree, no allocating
 * library routine).  Arguments, outputs and synchronisation as for
 * cl_sample_into; when m exceeds cap, m_out is set, edges holds the first cap
 * edges and the call returns CL_ERR_CAPACITY (call again with a larger
 * buffer: the array's plan is not reachable through cl_generate).
 * Limit: a plan whose workspace would exceed CL_NOALLOC_SCRATCH_BYTES (about
 * 32 bytes per source plus 9 to 10 bytes per edge: a power-law graph of
 * n = 1e5 with 2.7e6 edges needs 26.5 MB, so graphs up to about 6e6 edges
 * fit) returns CL_ERR_WORKSPACE, with the bytes it would need in
 * ws_required, before any edge is generated; edges are then untouched.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind (each call starts by resetting what must start at zero): calls
 * that overlap on one GPU (concurrent streams or host threads) race and
 * give undefined results; serialise them.
 * ------------------------------------------------------------------------- */
#define CL_NOALLOC_SCRATCH_BYTES (64ull << 20)
cl_status cl_sample_into_noalloc(const cl_graph* g /* host, G entries */, uint32_t G, const cl_tuning* t,
                                 uint32_t* edges, uint64_t cap, uint64_t* graph_offsets,
                                 uint64_t* m_out /* host */, uint64_t* ws_required /* host, may be NULL */,
                                 void* stream);

/* ---------------------------------------------------------------------------
 * Generation, write pass: the output E of Create-Edges (Sec. 3, Alg. 1) for
 * every planned task.  For a plan of cl_count, replays the planned lanes
 * with the same random words; for a plan of cl_sample, expands the lanes'
 * slot words (and replays the lanes whose slot overflowed).  Either way it
 * writes every edge whose position in the batch output lies in
 * [edge_begin, edge_begin + cap) to edges[2 (pos - edge_begin) + {0,1}] as
 * (u, v).  Task g's edges occupy positions [off_g, off_g + m_g), off_g = sum of
 * m_h for h < g.  graph_offsets (device, G + 1 entries, may be NULL) receives
 * off_0..off_{G-1} and the total.  Writing the output in windows (slabs)
 * costs each window only the lanes that overlap it (the windows are a
 * project addition: they stream an output larger than one buffer, and the
 * storage of a window is left out of the generation time, as Sec. 5 leaves
 * out I/O).  Asynchronous.
 * Precondition: ws holds the plan of a successful cl_count, cl_sample or
 * cl_sample_into (same inputs, unchanged).  The call does not read the plan
 * back, so it cannot report a workspace that holds no such plan: on a plan
 * of cl_plan (no counts), or a failed plan, its kernels return at once and
 * nothing is written.  cl_plan_info reports the state of a workspace.
 * ------------------------------------------------------------------------- */
cl_status cl_generate(void* ws, const cl_tuning* t, uint32_t* edges, uint64_t edge_begin, uint64_t cap,
                      uint64_t* graph_offsets, void* stream);

/* ---------------------------------------------------------------------------
 * The same edges as compressed sparse rows (the generator's output consumed
 * on the fly, as Sec. 4 suggests for analysis without disk I/O): col[pos] = v for the edge (u, v) at batch position pos
 * (4 bytes per edge instead of 8), and row_ptr[q_g + u] = the batch position
 * of the first edge of source u of task g, q_g = sum over earlier tasks h of
 * (n_h + 1), so that the targets of u are col[row_ptr[q_g + u] ..
 * row_ptr[q_g + u + 1]) and row_ptr[q_g + n_g] = off_g + m_g.  Rows of sources
 * outside the task's range are empty.  col: device uint32, cap >= total m;
 * row_ptr: device uint64, row_len >= sum_g (n_g + 1); else CL_ERR_CAPACITY.
 * ws must hold the plan of a successful cl_count, cl_sample or
 * cl_sample_into.  Synchronises once (reads the plan's sizes), then
 * launches asynchronously.
 * ------------------------------------------------------------------------- */
cl_status cl_generate_csr(void* ws, const cl_tuning* t, uint32_t* col, uint64_t cap, uint64_t* row_ptr,
                          uint64_t row_len, void* stream);

/* ---------------------------------------------------------------------------
 * The plan alone (validation, quantised prefix, segments, lane plan), without
 * running the lanes: for cl_degrees, which needs no counts.  ws as for
 * cl_count (cl_workspace_size with one_pass = 0 bounds it).  cl_generate on
 * such a workspace writes nothing.  Synchronises twice.
 * ------------------------------------------------------------------------- */
cl_status cl_plan(const cl_graph* g /* host, G entries */, uint32_t G, const cl_tuning* t, void* ws,
                  uint64_t ws_bytes, uint64_t* ws_required /* host, may be NULL */, void* stream);

/* ---------------------------------------------------------------------------
 * Degrees of the planned graphs without storing any edge (the generator's
 * output analysed on the fly, which Sec. 4 names as a use of generation
 * without disk I/O):
 * runs the planned lanes once more with the same random words and adds, for
 * every kept edge (u, v), 1 to deg[q_g + u] and deg[q_g + v], where
 * q_g = sum over earlier tasks h of (n_h + 1) (for one task, deg[0 .. n)).
 * Adds into deg (the caller zeroes it, so that several plans, e.g. the parts
 * of a partition, can accumulate into one array).  deg: device uint32,
 * deg_len >= sum_g (n_g + 1), else CL_ERR_CAPACITY.  ws must hold a plan of
 * cl_count, cl_sample or cl_plan.  Synchronises once (reads the plan's
 * sizes), then launches asynchronously.
 * ------------------------------------------------------------------------- */
cl_status cl_degrees(void* ws, const cl_tuning* t, uint32_t* deg, uint64_t deg_len, void* stream);

/* ---------------------------------------------------------------------------
 * Work-unit statistics of a plan, for Sec. 4's comparison of partitions
 * (runtime of a part against its cost c(V_i) = m_i + |V_i|, Eq. 2-4; the
 * imbalance of the naive consecutive and the round-robin partitions): runs
 * the planned lanes once more as a count pass (the same candidates; no
 * output; the plan's counts are rewritten with the same values) and records
 * for every work unit i four 64-bit words at stats[4 i]:
 *   [0] wave clock (s_memrealtime, 100 MHz) when a lane took the unit,
 *   [1] wave clock when it finished it,
 *   [2] low 32 bits: the unit's plan cost (the sum over its segments of
 *       c_u / K_u, in cost units of 1/16 expected candidate, rounded);
 *       high 32 bits: the candidates it visited,
 *   [3] low 32 bits: its edges; high 32 bits: the lane that ran it
 *       (wavefront index * 64 + lane).
 * Every unit gets a record; the units of the padding to whole wavefronts
 * carry no segments (cost, candidates and edges 0).
 * ws: a plan of cl_count, cl_sample or cl_plan (any partition policy).
 * stats: device, stats_len >= 4 x units (units_out, host, may be NULL, gets
 * the number of units), else CL_ERR_CAPACITY with nothing launched (stats
 * may be NULL with stats_len 0 to ask for the size).  Synchronises once (reads the
 * plan's sizes), then launches asynchronously.  A project addition for
 * measurement; it does not change any output.
 * ------------------------------------------------------------------------- */
cl_status cl_unit_stats(void* ws, const cl_tuning* t, uint64_t* stats, uint64_t stats_len,
                        uint64_t* units_out /* host, may be NULL */, void* stream);

/* Totals of the plan in ws (host outputs, each may be NULL; synchronises).
 * lanes includes the padding to whole wavefronts; candidates is the number of
 * candidates the lane kernel visited (the edge-plus-source work of Eq. 2-4,
 * rejections included); lane_kernel_ms is the duration of that kernel
 * (count pass or one pass), timed by HIP events on the caller's stream and
 * stored on that stream after the planning call returns (read it there);
 * overflow_lanes counts one-pass lanes that exceeded their slot; slot_words
 * is the number of 32-bit words the one pass needed for its slots (one per
 * edge plus two per change of source inside a lane; 0 for other plans). */
cl_status cl_plan_info(const void* ws, uint64_t* lanes, uint64_t* heavy_segments, uint64_t* edges,
                       uint64_t* candidates, float* lane_kernel_ms, uint32_t* overflow_lanes,
                       uint64_t* slot_words, void* stream);

/* ---------------------------------------------------------------------------
 * Digest of an edge list: acc += sum_i mix(mix(index_base + i) ^ (u_i 2^32 + v_i))
 * mod 2^64, mix = splitmix64's output function.  Order independent
 * reduction, position keyed.  acc: device uint64 the caller initialises.
 * Asynchronous.
 * ------------------------------------------------------------------------- */
cl_status cl_hash_edges(const uint32_t* edges, uint64_t m, uint64_t index_base, uint64_t* acc, void* stream);

/* ---------------------------------------------------------------------------
 * Batched generation as one replayable HIP graph (a project addition: each
 * of the G tasks is Create-Edges(w, S, V) of Sec. 3, Alg. 1, and the batch
 * output is their concatenation, as from G calls): records the whole path
 * (validation, prefix, plan, count or one pass, offsets, output) for the G
 * tasks planned in ws by a preceding cl_count or cl_sample (same g), with the
 * sizes of that plan, on a
 * non-null stream in capture mode.  Each replay regenerates all G edge lists
 * into edges[0 .. 2 cap) with no host synchronisation; graph_offsets (device,
 * G + 1) receives the task offsets.  If a replay finds larger sizes than the
 * plan (changed inputs) it writes nothing and cl_plan_info reports 0 edges.
 * A workspace that holds no counted plan (none, a failed one, or one of
 * cl_plan) gives CL_ERR_NOT_PLANNED and nothing is captured.
 * ------------------------------------------------------------------------- */
cl_status cl_batch_capture(const cl_graph* g /* host */, uint32_t G, const cl_tuning* t, void* ws,
                           uint32_t* edges, uint64_t cap, uint64_t* graph_offsets,
                           void** graph_exec_out /* host */, void* stream);
cl_status cl_batch_launch(void* graph_exec, void* stream);
cl_status cl_batch_destroy(void* graph_exec);

/* ---------------------------------------------------------------------------
 * Expected degrees under the capped model (Sec. 3, with j != i and the cap):
 *   d_i = sum_{j != i} min(w_i w_j / S, 1).
 * w: float32, non-negative (any order).  Pair terms in float32, accumulated in float32 over
 * tiles of columns; tile partials summed in float64.  d_out: float64.
 * ws: cl_expected_degree_workspace bytes.  Asynchronous.
 * ------------------------------------------------------------------------- */
cl_status cl_expected_degree_workspace(uint64_t n, uint64_t* bytes_out /* host */);
cl_status cl_expected_degree(const float* w, uint64_t n, double S, double* d_out, void* ws, uint64_t ws_bytes,
                             const cl_tuning* t /* tile shape; NULL = defaults */, void* stream);

/* Adjoint of cl_expected_degree: given g = dL/dd (float64), writes
 *   grad_w[k] = (g_k A_k + B_k - T) / S,  A_k = sum_{j != k, x_kj < 1} w_j,
 *   B_k = sum_{j != k, x_kj < 1} g_j w_j,  T = sum_i g_i sum_{j != i, x_ij < 1} x_ij,
 * x_ij = w_i w_j / S; the T term (dS/dw_k = 1) only when s_depends_on_w != 0.
 * Pairs with x_ij >= 1 are capped (zero derivative).  grad_w: float32.
 * Asynchronous. */
cl_status cl_expected_degree_backward(const float* w, uint64_t n, double S, const double* grad_d,
                                      int s_depends_on_w, float* grad_w, void* ws, uint64_t ws_bytes,
                                      const cl_tuning* t /* tile shape; NULL = defaults */, void* stream);

/* Number of compute units of the current device (host; 0 on error). */
uint32_t cl_device_cus(void);

/* Version string of the library (host, static storage). */
const char* cl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CLGEN_H_ */
