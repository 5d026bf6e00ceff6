// C ABI of the generator (declarations and contracts in include/clgen.h).
// Host side only: argument checks, workspace layout, launches.  Every step of
// the computation runs in the kernels of cl_kernels.hpp, cl_stats.hpp and
// cl_expdeg.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "clgen.h"
#include "cl_expdeg.hpp"
#include "cl_kernels.hpp"
#include "cl_order.hpp"
#include "cl_plan.hpp"
#include "cl_scan.hpp"
#include "cl_stats.hpp"

using namespace cl;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint32_t kDefaultBudget = 192;
constexpr uint32_t kDefaultBlocksPerCu = 3;
constexpr int kPersistThreads = 256;
unsigned long long* const kNoRows = nullptr;   // row counts: CSR output only
UnitStat* const kNoStats = nullptr;            // unit records: statistics pass only
static_assert(kPersistThreads == kLaneThreads, "the lane kernels stage output for 256 threads");

inline uint64_t align_up(uint64_t x, uint64_t a = kAlign) { return (x + a - 1) / a * a; }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline cl_status hip_status(hipError_t e) { return e == hipSuccess ? CL_OK : CL_ERR_DEVICE; }

#define CL_TRY(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return CL_ERR_DEVICE;        \
  } while (0)

uint32_t cus_of_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return static_cast<uint32_t>(cus);
}

cl_status status_error(uint32_t st) {
  if (st & kStNonfinite) return CL_ERR_NONFINITE;
  if (st & kStNegative) return CL_ERR_NEGATIVE;
  if (st & kStUnsorted) return CL_ERR_UNSORTED;
  if (st & kStBadS) return CL_ERR_INVALID_ARG;
  if (st & kStCapacity) return CL_ERR_CAPACITY;
  if (st & kStCostOverflow) return CL_ERR_TOO_LARGE;
  return st ? CL_ERR_DEVICE : CL_OK;
}

uint32_t grid_for(uint64_t items, uint32_t threads, uint32_t cap_blocks) {
  uint64_t b = (items + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return static_cast<uint32_t>(b);
}

uint32_t stream_grid_cap() {
  const uint32_t cus = cus_of_current_device();
  return std::max<uint32_t>(cus, 1) * 16;
}

bool finite_pos(double x) { return x > 0.0 && x <= 1.7976931348623157e308; }

// ---------------------------------------------------------------- layouts
struct FixedLayout {
  uint64_t off_desc, off_Q, off_C, off_SB, off_A, off_scan, off_m, bytes;
  uint64_t total_q, total_r, scan_elems;
};

FixedLayout fixed_layout(const cl_graph* g, uint32_t G) {
  FixedLayout L{};
  uint64_t tq = 0, tr = 0;
  for (uint32_t i = 0; i < G; ++i) {
    tq += g[i].n + 1;
    tr += (g[i].u_end - g[i].u_begin) + 1;
  }
  L.total_q = tq;
  L.total_r = tr;
  // scan partials: Triple tiles of the source scan or u64 tiles of the Q scan
  L.scan_elems = std::max<uint64_t>(scan_tiles(tq), 3 * scan_tiles<Triple>(tr)) + 8;
  // the edge counts follow the header, so that one copy reads both back
  uint64_t off = align_up(sizeof(WsHeader));
  L.off_m = off;
  off = align_up(off + 8 * G);
  L.off_desc = off;
  off = align_up(off + sizeof(GraphDesc) * G);
  L.off_Q = off;
  off = align_up(off + 8 * tq);
  L.off_C = off;
  off = align_up(off + 8 * tr);
  L.off_SB = off;
  off = align_up(off + 8 * tr);
  L.off_A = off;
  off = align_up(off + 8 * tr);
  L.off_scan = off;
  off = align_up(off + 8 * L.scan_elems);
  L.bytes = off;
  return L;
}

struct VarLayout {
  uint64_t off_hseg, off_lstart, off_lcnt, off_lpos, off_lscan, off_groups, bytes;
  uint64_t off_lcum, off_soff, off_sscan, off_lwords, off_slots, slot_cap;
  uint64_t off_perm, off_ohist, off_okeys, oblocks;
};

// nh heavy segments, nl lanes; with one_pass, slot_cap words of slots; with
// ordered, the processing order of the units and its count matrix
VarLayout var_layout(uint64_t base, uint64_t nh, uint64_t nl, bool one_pass, uint64_t slot_cap,
                     bool ordered = false) {
  VarLayout V{};
  uint64_t off = align_up(base);
  V.off_hseg = off;
  off = align_up(off + sizeof(HSeg) * std::max<uint64_t>(nh, 1));
  V.off_lstart = off;
  off = align_up(off + 4 * std::max<uint64_t>(nl, 1));
  V.off_lcnt = off;
  off = align_up(off + 4 * std::max<uint64_t>(nl, 1));
  V.off_lpos = off;
  off = align_up(off + 8 * (nl + 1));
  V.off_lscan = off;
  off = align_up(off + 8 * (scan_tiles(nl + 1) + 8));
  V.off_groups = off;
  off = align_up(off + 4 * std::max<uint64_t>(nl / kLaneGroup, 1));
  if (one_pass) {
    V.off_lcum = off;
    off = align_up(off + 8 * (nl + 1));
    V.off_soff = off;
    off = align_up(off + 8 * (nl + 1));
    V.off_sscan = off;
    off = align_up(off + 8 * (scan_tiles(nl + 1) + 8));
    V.off_lwords = off;
    off = align_up(off + 4 * std::max<uint64_t>(nl, 1));
    V.off_slots = off;
    V.slot_cap = slot_cap;
    off = align_up(off + 4 * std::max<uint64_t>(slot_cap, 1));
  }
  if (ordered) {
    V.oblocks = order_blocks(nl);
    V.off_perm = off;
    off = align_up(off + 4 * std::max<uint64_t>(nl, 1));
    V.off_ohist = off;
    off = align_up(off + 4 * (2 * kOrderBins + 2));
    V.off_okeys = off;
    off = align_up(off + 2 * std::max<uint64_t>(nl, 1));
  }
  V.bytes = off;
  return V;
}

// upper bound of the slot capacities in words: sum (mu + 8 sqrt(mu) + 25 +
// 2 segments + 15 of rounding) over the lanes, with sum sqrt(mu) <=
// sqrt(lanes * sum mu)
uint64_t slot_bound(uint64_t total_cost, uint64_t nl, uint64_t nseg) {
  const double mu = static_cast<double>(total_cost) / kCostUnit;
  const double b = mu + 8.0 * std::sqrt(static_cast<double>(nl) * mu) + 40.0 * static_cast<double>(nl) +
                   2.0 * static_cast<double>(nseg) + 64.0;
  return static_cast<uint64_t>(std::ceil(b));
}

cl_status check_graphs(const cl_graph* g, uint32_t G) {
  if (!g || G == 0) return CL_ERR_INVALID_ARG;
  for (uint32_t i = 0; i < G; ++i) {
    if (g[i].n >= 4294967296ull) return CL_ERR_TOO_LARGE;
    if (g[i].n > 0 && g[i].w == nullptr) return CL_ERR_INVALID_ARG;
    if (!finite_pos(g[i].S)) return CL_ERR_INVALID_ARG;
    if (g[i].u_begin > g[i].u_end || g[i].u_end > g[i].n) return CL_ERR_INVALID_ARG;
  }
  return CL_OK;
}

// processing order of a plan's units: 1 = index order, 2 = by position
// (cl_tuning.unit_order; 0 takes 2 for a single graph, 1 for a batch)
constexpr uint32_t kOrderRefused = 0xFFFFFFFFu;
uint32_t ordered_units(const cl_tuning* t, uint32_t G) {
  const uint32_t o = t ? t->unit_order : 0u;
  if (o == 0) return (G == 1) ? 2u : 1u;
  if (o > 2 || (o == 2 && G != 1)) return kOrderRefused;
  return o;
}

uint64_t budget_units(const cl_tuning* t) {
  const uint32_t b = (t && t->lane_budget) ? t->lane_budget : kDefaultBudget;
  return static_cast<uint64_t>(b) * kCostUnit;
}

uint32_t persistent_grid(const cl_tuning* t) {
  const uint32_t bpc = (t && t->blocks_per_cu) ? t->blocks_per_cu : kDefaultBlocksPerCu;
  return std::max<uint32_t>(cus_of_current_device(), 1) * bpc;
}

// the phase of the plan that needs no sizes from the device: validation,
// quantised prefix, per-source prefixes, per-graph sizes
hipError_t launch_plan_front(WsHeader* dhdr, const WsHeader& h, uint32_t G, hipStream_t s) {
  const uint32_t cap = stream_grid_cap();
  hipLaunchKernelGGL(k_plan_init, dim3((G + 255) / 256), dim3(256), 0, s, dhdr);
  hipLaunchKernelGGL((k_validate<false>), dim3(grid_for(h.total_q, 256, cap)), dim3(256), 0, s, h.desc, G,
                     h.total_q, kNoRows);
  hipError_t e = device_scan<uint64_t>(QIn{h.desc, G}, QOut{h.desc, G, h.Q}, h.total_q, h.scan_tmp, s);
  if (e != hipSuccess) return e;
  e = device_scan<Triple>(NodeIn{h.desc, G, h.Q}, NodeOut{h.desc, G, h.C, h.SB}, h.total_r,
                          reinterpret_cast<Triple*>(h.scan_tmp), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plan_sizes, dim3(1), dim3(256), 0, s, dhdr);
  return hipGetLastError();
}

// the rest: heavy table, lane plan, then either the count pass (two-pass
// plans) or the one pass into slots, and the offsets
hipError_t launch_plan_back(WsHeader* dhdr, const WsHeader& h, const cl_tuning* t, hipStream_t s,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  const uint32_t cap = stream_grid_cap();
  hipLaunchKernelGGL(k_heavy_table, dim3(grid_for(h.cap_nh, 256, cap)), dim3(256), 0, s, dhdr);
  hipLaunchKernelGGL(k_lane_plan, dim3(grid_for(h.total_r, 256, cap)), dim3(256), 0, s, dhdr);
  hipLaunchKernelGGL(k_lane_groups, dim3(grid_for(h.cap_nl, 256, cap)), dim3(256), 0, s, dhdr);
  {
    hipError_t e = launch_order(dhdr, h, s);   // processing order of the units, if asked for
    if (e != hipSuccess) return e;
  }
  // (the unit queue and the overflow count were cleared with the status)
  if (h.mode == 2) {   // plan only (cl_plan): no lane kernel, no counts
    if (ev0) (void)hipEventRecord(ev0, s);
    if (ev1) (void)hipEventRecord(ev1, s);
    return hipGetLastError();
  }
  if (h.mode == 1) {
    hipError_t e = device_scan<uint64_t>(SlotIn{dhdr}, SlotOut{{}, h.slot_off, h.slot_cap, dhdr}, h.cap_nl + 1,
                                         h.slot_scan_tmp, s);   // also checks the total against the capacity
    if (e != hipSuccess) return e;
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL((k_lanes<2>), dim3(persistent_grid(t)), dim3(kPersistThreads), 0, s, dhdr,
                       static_cast<uint2*>(nullptr), 0ull, 0ull, static_cast<uint32_t*>(nullptr), kNoRows, kNoStats);
    if (ev1) (void)hipEventRecord(ev1, s);
  } else {
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL((k_lanes<0>), dim3(persistent_grid(t)), dim3(kPersistThreads), 0, s, dhdr,
                       static_cast<uint2*>(nullptr), 0ull, 0ull, static_cast<uint32_t*>(nullptr), kNoRows, kNoStats);
    if (ev1) (void)hipEventRecord(ev1, s);
  }
  hipError_t e = device_scan<uint64_t>(CntIn{{}, h.lane_cnt, h.cap_nl}, OffOut{{}, h.lane_pos}, h.cap_nl + 1,
                                       h.lane_scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_graph_edges, dim3(grid_for(h.G, 256, cap)), dim3(256), 0, s, dhdr, h.m_dev);
  return hipGetLastError();
}

// output of a planned workspace into the window [lo, hi): compaction of the
// slots (one-pass plans) and the replay kernel (every lane for two-pass plans,
// only overflowed lanes for one-pass plans); each kernel returns at once when
// the plan is not of its kind
hipError_t launch_write(WsHeader* dhdr, const cl_tuning* t, uint32_t* edges, uint64_t lo, uint64_t hi,
                        uint64_t* graph_offsets, hipStream_t s) {
  const uint32_t cus = std::max<uint32_t>(cus_of_current_device(), 1);
  hipLaunchKernelGGL((k_compact<false>), dim3(cus * 16), dim3(256), 0, s, dhdr, reinterpret_cast<uint2*>(edges), lo,
                     hi, kNoRows);   // also clears the unit queue
  hipLaunchKernelGGL((k_lanes<1>), dim3(persistent_grid(t)), dim3(kPersistThreads), 0, s, dhdr,
                     reinterpret_cast<uint2*>(edges), lo, hi, static_cast<uint32_t*>(nullptr), kNoRows, kNoStats);
  if (graph_offsets) hipLaunchKernelGGL(k_graph_offsets, dim3(16), dim3(256), 0, s, dhdr, graph_offsets);
  return hipGetLastError();
}

}  // namespace

extern "C" {

const char* cl_version(void) { return "clgen 1.0 (gfx950)"; }

uint32_t cl_device_cus(void) { return cus_of_current_device(); }

// ------------------------------------------------------------ exact sum
cl_status cl_weight_sum_workspace(uint64_t n, uint64_t* bytes_out) {
  (void)n;
  if (!bytes_out) return CL_ERR_INVALID_ARG;
  *bytes_out = align_up(sizeof(GraphDesc)) + align_up(16ull * kBins) + kAlign;
  return CL_OK;
}

cl_status cl_weight_sum(const double* w, uint64_t n, void* ws, uint64_t ws_bytes, double* S_out, void* stream) {
  if (!S_out || (n > 0 && !w)) return CL_ERR_INVALID_ARG;
  if (n >= 4294967296ull) return CL_ERR_TOO_LARGE;
  uint64_t need = 0;
  cl_weight_sum_workspace(n, &need);
  if (!ws || ws_bytes < need) return CL_ERR_WORKSPACE;
  if (n == 0) {
    *S_out = 0.0;
    return CL_OK;
  }
  hipStream_t s = as_stream(stream);
  char* base = static_cast<char*>(ws);
  GraphDesc* d = reinterpret_cast<GraphDesc*>(base);
  unsigned long long* bins = reinterpret_cast<unsigned long long*>(base + align_up(sizeof(GraphDesc)));
  double* S_dev = reinterpret_cast<double*>(base + align_up(sizeof(GraphDesc)) + align_up(16ull * kBins));
  GraphDesc h{};
  h.w = w;
  h.n = n;
  h.S = __builtin_inf();
  h.q_off = 0;
  CL_TRY(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero_u64, dim3(16), dim3(256), 0, s, bins, static_cast<uint64_t>(2 * kBins));
  // few blocks: every block adds its nonzero bins to the same few global words
  const uint32_t cap = std::max<uint32_t>(cus_of_current_device(), 1) * 4;
  hipLaunchKernelGGL((k_validate<true>), dim3(grid_for(n + 1, 256, cap)), dim3(256), 0, s, d, 1u, n + 1, bins);
  hipLaunchKernelGGL(k_sum_finalize, dim3(1), dim3(64), 0, s, bins, S_dev, &d->status);
  CL_TRY(hipGetLastError());
  // S and the status word, stored side by side by the finaliser: one read-back
  uint64_t res[2] = {0, 0};
  CL_TRY(hipMemcpyAsync(res, S_dev, sizeof(res), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  double Sh;
  memcpy(&Sh, &res[0], sizeof(Sh));
  uint32_t st = static_cast<uint32_t>(res[1]);
  st &= ~static_cast<uint32_t>(kStBadS);   // no S given: the w_0 / S conditions do not apply
  if (st) return status_error(st);
  *S_out = Sh;
  return CL_OK;
}

// ------------------------------------------------------- expected edges
cl_status cl_expected_edges_workspace(uint64_t n, uint64_t* bytes_out) {
  if (!bytes_out) return CL_ERR_INVALID_ARG;
  const uint64_t nt = scan_tiles(n + 1);
  *bytes_out = align_up(16 * (n + 1)) + align_up(16 * (nt + 8)) + align_up(16 * 4096) + align_up(16);
  return CL_OK;
}

cl_status cl_expected_edges(const double* w, uint64_t n, double S, void* ws, uint64_t ws_bytes, double* Em_out,
                            double* Var_out, void* stream) {
  if (!Em_out || !Var_out || (n > 0 && !w) || !finite_pos(S)) return CL_ERR_INVALID_ARG;
  if (n >= 4294967296ull) return CL_ERR_TOO_LARGE;
  uint64_t need = 0;
  cl_expected_edges_workspace(n, &need);
  if (!ws || ws_bytes < need) return CL_ERR_WORKSPACE;
  if (n == 0) {
    *Em_out = 0.0;
    *Var_out = 0.0;
    return CL_OK;
  }
  hipStream_t s = as_stream(stream);
  char* base = static_cast<char*>(ws);
  const uint64_t nt = scan_tiles(n + 1);
  Dbl2* suf = reinterpret_cast<Dbl2*>(base);
  Dbl2* scan_tmp = reinterpret_cast<Dbl2*>(base + align_up(16 * (n + 1)));
  Dbl2* parts = reinterpret_cast<Dbl2*>(base + align_up(16 * (n + 1)) + align_up(16 * (nt + 8)));
  Dbl2* out = reinterpret_cast<Dbl2*>(base + align_up(16 * (n + 1)) + align_up(16 * (nt + 8)) + align_up(16 * 4096));
  CL_TRY((device_scan<Dbl2>(SufIn{{}, w, n}, SufOut{{}, suf, n}, n + 1, scan_tmp, s)));
  const uint32_t nb = grid_for(n, 256, 4096);
  hipLaunchKernelGGL(k_expected_edges, dim3(nb), dim3(256), 0, s, w, n, S, suf, parts);
  hipLaunchKernelGGL(k_reduce_dbl2, dim3(1), dim3(256), 0, s, parts, nb, out);
  CL_TRY(hipGetLastError());
  Dbl2 h{};
  CL_TRY(hipMemcpyAsync(&h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  *Em_out = h.a;
  *Var_out = h.b;
  return CL_OK;
}

// ------------------------------------------------------------ partition
cl_status cl_partition_workspace(uint64_t n, uint32_t P, uint64_t* bytes_out) {
  if (!bytes_out) return CL_ERR_INVALID_ARG;
  *bytes_out = align_up(sizeof(GraphDesc)) + align_up(8 * (n + 1)) * 2 + align_up(8 * (scan_tiles(n + 1) + 8)) +
               align_up(8 * (static_cast<uint64_t>(P) + 1));
  return CL_OK;
}

cl_status cl_partition(const double* w, uint64_t n, double S, uint32_t P, void* ws, uint64_t ws_bytes,
                       uint64_t* bounds_out, uint64_t* total_cost_out, void* stream) {
  if (!bounds_out || P == 0 || P > (1u << 24) || (n > 0 && !w) || !finite_pos(S)) return CL_ERR_INVALID_ARG;
  if (n >= 4294967296ull) return CL_ERR_TOO_LARGE;
  uint64_t need = 0;
  cl_partition_workspace(n, P, &need);
  if (!ws || ws_bytes < need) return CL_ERR_WORKSPACE;
  if (n == 0) {
    for (uint32_t k = 0; k <= P; ++k) bounds_out[k] = 0;
    if (total_cost_out) *total_cost_out = 0;
    return CL_OK;
  }
  hipStream_t s = as_stream(stream);
  char* base = static_cast<char*>(ws);
  GraphDesc* d = reinterpret_cast<GraphDesc*>(base);
  uint64_t off = align_up(sizeof(GraphDesc));
  uint64_t* Q = reinterpret_cast<uint64_t*>(base + off);
  off += align_up(8 * (n + 1));
  uint64_t* C = reinterpret_cast<uint64_t*>(base + off);
  off += align_up(8 * (n + 1));
  uint64_t* tmp = reinterpret_cast<uint64_t*>(base + off);
  off += align_up(8 * (scan_tiles(n + 1) + 8));
  uint64_t* bd = reinterpret_cast<uint64_t*>(base + off);
  GraphDesc h{};
  h.w = w;
  h.n = n;
  h.S = S;
  h.u_begin = 0;
  h.u_end = n;
  CL_TRY(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, s));
  const uint32_t cap = stream_grid_cap();
  hipLaunchKernelGGL(k_graph_init, dim3(1), dim3(64), 0, s, d, 1u);
  hipLaunchKernelGGL((k_validate<false>), dim3(grid_for(n + 1, 256, cap)), dim3(256), 0, s, d, 1u, n + 1,
                     kNoRows);
  CL_TRY((device_scan<uint64_t>(QIn{d, 1u}, QOut{d, 1u, Q}, n + 1, tmp, s)));
  CL_TRY((device_scan<uint64_t>(PartIn{{}, d, Q}, PartOut{{}, C}, n + 1, tmp, s)));
  hipLaunchKernelGGL(k_part_bounds, dim3(grid_for(static_cast<uint64_t>(P) + 1, 256, 1024)), dim3(256), 0, s, C, n,
                     P, bd);
  CL_TRY(hipGetLastError());
  uint32_t st = 0;
  uint64_t Z = 0;
  CL_TRY(hipMemcpyAsync(bounds_out, bd, 8 * (static_cast<uint64_t>(P) + 1), hipMemcpyDeviceToHost, s));
  CL_TRY(hipMemcpyAsync(&st, &d->status, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CL_TRY(hipMemcpyAsync(&Z, C + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  if (st) return status_error(st);
  if (total_cost_out) *total_cost_out = Z;
  return CL_OK;
}

// ----------------------------------------------------------- generation
cl_status cl_workspace_size(const cl_graph* g, uint32_t G, const cl_tuning* t, uint32_t one_pass,
                            uint64_t* fixed_bytes, uint64_t* estimate_bytes) {
  cl_status st = check_graphs(g, G);
  if (st != CL_OK) return st;
  if (ordered_units(t, G) == kOrderRefused) return CL_ERR_INVALID_ARG;
  const FixedLayout F = fixed_layout(g, G);
  // estimate (when S = sum w): expected edges <= S/2, plan cost ~ 16 (S/2 + 2 range),
  // heavy segments ~ S/256
  const uint64_t bu = budget_units(t) / kCostUnit;
  double nl = 0.0, nh = 0.0, cost = 0.0, nseg = 0.0;
  for (uint32_t i = 0; i < G; ++i) {
    const double nr = static_cast<double>(g[i].u_end - g[i].u_begin);
    nl += 1.5 * (g[i].S * 0.5 + 2.0 * nr) / static_cast<double>(bu) + kLaneGroup;   // graded tail: up to +38 %
    nh += g[i].S / 256.0 + 64.0;
    nseg += g[i].S / 256.0 + 64.0 + nr;
    cost += kCostUnit * (g[i].S * 0.5 + 2.0 * nr);
  }
  const uint64_t nl64 = static_cast<uint64_t>(nl) / kLaneGroup * kLaneGroup + kLaneGroup * G;
  const VarLayout V = var_layout(F.bytes, static_cast<uint64_t>(nh), nl64, one_pass != 0,
                                 one_pass ? slot_bound(static_cast<uint64_t>(cost), nl64, static_cast<uint64_t>(nseg)) : 0,
                                 ordered_units(t, G) == 2);
  if (fixed_bytes) *fixed_bytes = F.bytes;
  if (estimate_bytes) *estimate_bytes = V.bytes;
  return CL_OK;
}

// mode 0: plan + count pass; 1: plan + one pass into slots; 2: plan only.
// With `into` (mode 1), the expansion into edges[0, cap) and graph_offsets is
// queued before the final read-back.
struct IntoOut {
  uint32_t* edges;
  uint64_t cap;
  uint64_t* graph_offsets;
};

// The pair of events that times the lane kernel: created once per thread
// and device and reused by every plan on them (a plan synchronises its
// stream before reading the pair, so no record is pending at the next one).
// Both null if they cannot be created.
static void lane_events(hipEvent_t* e0, hipEvent_t* e1) {
  static thread_local std::vector<std::pair<hipEvent_t, hipEvent_t>> cache;
  *e0 = nullptr;
  *e1 = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    (void)hipGetLastError();
    return;
  }
  if (cache.size() <= static_cast<size_t>(dev)) cache.resize(static_cast<size_t>(dev) + 1, {nullptr, nullptr});
  auto& p = cache[static_cast<size_t>(dev)];
  if (!p.first) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      (void)hipGetLastError();
      return;
    }
    p = {a, b};
  }
  *e0 = p.first;
  *e1 = p.second;
}

static cl_status plan_common(const cl_graph* g, uint32_t G, const cl_tuning* t, void* ws, uint64_t ws_bytes,
                             uint64_t* m_out, uint64_t* ws_required, void* stream, uint32_t mode,
                             const IntoOut* into = nullptr) {
  cl_status st = check_graphs(g, G);
  if (st != CL_OK) return st;
  if (!m_out) return CL_ERR_INVALID_ARG;
  const uint32_t policy = t ? t->partition : 0u;
  // round-robin units do not produce (u, v)-ordered runs: plan only
  if (policy > 2 || (policy == 2 && mode != 2)) return CL_ERR_INVALID_ARG;
  // a processing order by position: single-graph plans (a chunk of units
  // never spans two graphs); the default for them
  const uint32_t order = ordered_units(t, G);
  if (order == kOrderRefused) return CL_ERR_INVALID_ARG;
  const FixedLayout F = fixed_layout(g, G);
  if (ws_required) *ws_required = F.bytes;
  if (!ws || ws_bytes < F.bytes) return CL_ERR_WORKSPACE;
  hipStream_t s = as_stream(stream);
  char* base = static_cast<char*>(ws);
  WsHeader* dhdr = reinterpret_cast<WsHeader*>(base);

  std::vector<GraphDesc> desc(G);
  uint64_t qo = 0, ro = 0;
  const uint64_t bu = budget_units(t);
  for (uint32_t i = 0; i < G; ++i) {
    GraphDesc d{};
    d.w = g[i].w;
    d.n = g[i].n;
    d.S = g[i].S;
    d.seed = g[i].seed;
    d.u_begin = g[i].u_begin;
    d.u_end = g[i].u_end;
    d.q_off = qo;
    d.r_off = ro;
    d.budget = bu;
    d.policy = policy;
    // graded units only for the last task: the work queue hands out the units
    // of the tasks in order, so only the last one's end leaves lanes idle
    d.graded = ((t && t->tail_units == 1) || i + 1 != G) ? 0u : 1u;
    qo += g[i].n + 1;
    ro += (g[i].u_end - g[i].u_begin) + 1;
    desc[i] = d;
  }
  WsHeader h{};
  h.magic = kWsMagic;
  h.G = G;
  h.total_q = F.total_q;
  h.total_r = F.total_r;
  h.cap_nh = 0;
  h.cap_nl = 0;
  h.bytes_fixed = F.bytes;
  h.desc = reinterpret_cast<GraphDesc*>(base + F.off_desc);
  h.Q = reinterpret_cast<uint64_t*>(base + F.off_Q);
  h.C = reinterpret_cast<uint64_t*>(base + F.off_C);
  h.SB = reinterpret_cast<uint64_t*>(base + F.off_SB);
  h.A = reinterpret_cast<double*>(base + F.off_A);
  h.scan_tmp = reinterpret_cast<uint64_t*>(base + F.off_scan);
  h.scan_tmp_elems = F.scan_elems;
  h.m_dev = reinterpret_cast<uint64_t*>(base + F.off_m);
  // header, edge counts (zero) and descriptors in one upload
  std::vector<unsigned char> up(F.off_desc + sizeof(GraphDesc) * G, 0);
  memcpy(up.data(), &h, sizeof(h));
  memcpy(up.data() + F.off_desc, desc.data(), sizeof(GraphDesc) * G);
  CL_TRY(hipMemcpyAsync(dhdr, up.data(), up.size(), hipMemcpyHostToDevice, s));
  CL_TRY(launch_plan_front(dhdr, h, G, s));
  WsHeader back{};
  CL_TRY(hipMemcpyAsync(&back, dhdr, sizeof(back), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  if (back.status) return status_error(back.status);

  const bool one_pass = (mode == 1);
  const VarLayout V = var_layout(F.bytes, back.total_nh, back.total_nl, one_pass,
                                 one_pass ? slot_bound(back.total_cost, back.total_nl, back.total_seg) : 0,
                                 order == 2);
  if (ws_required) *ws_required = V.bytes;
  if (ws_bytes < V.bytes) return CL_ERR_WORKSPACE;
  h.cap_nh = back.total_nh;
  h.cap_nl = back.total_nl;
  h.total_nh = back.total_nh;
  h.total_nl = back.total_nl;
  h.bytes_total = V.bytes;
  h.hseg = reinterpret_cast<HSeg*>(base + V.off_hseg);
  h.lane_seg = reinterpret_cast<uint32_t*>(base + V.off_lstart);
  h.lane_cnt = reinterpret_cast<uint32_t*>(base + V.off_lcnt);
  h.lane_pos = reinterpret_cast<uint64_t*>(base + V.off_lpos);
  h.lane_scan_tmp = reinterpret_cast<uint64_t*>(base + V.off_lscan);
  h.group_graph = reinterpret_cast<uint32_t*>(base + V.off_groups);
  h.mode = mode;
  h.overflow = 0;
  h.slot_margin = (t && t->slot_margin == 1) ? 1u : 0u;
  if (one_pass) {
    h.lane_cum = reinterpret_cast<uint64_t*>(base + V.off_lcum);
    h.slot_off = reinterpret_cast<uint64_t*>(base + V.off_soff);
    h.slot_scan_tmp = reinterpret_cast<uint64_t*>(base + V.off_sscan);
    h.lane_words = reinterpret_cast<uint32_t*>(base + V.off_lwords);
    h.slots = reinterpret_cast<uint32_t*>(base + V.off_slots);
    h.slot_cap = V.slot_cap;
  } else {
    h.lane_words = nullptr;
    h.lane_cum = nullptr;
    h.slot_off = nullptr;
    h.slot_scan_tmp = nullptr;
    h.slots = nullptr;
    h.slot_cap = 0;
  }
  if (order == 2) {
    h.perm = reinterpret_cast<uint32_t*>(base + V.off_perm);
    h.order_hist = reinterpret_cast<uint32_t*>(base + V.off_ohist);
    h.order_keys = reinterpret_cast<uint16_t*>(base + V.off_okeys);
    h.order_blocks = V.oblocks;
  } else {
    h.perm = nullptr;
    h.order_hist = nullptr;
    h.order_keys = nullptr;
    h.order_blocks = 0;
  }
  h.status = 0;
  h.queue = 0;
  h.planned = 0;
  CL_TRY(hipMemcpyAsync(dhdr, &h, sizeof(h), hipMemcpyHostToDevice, s));
  // the lane kernel is timed with HIP events on the caller's stream
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  lane_events(&ev0, &ev1);
  // planned: 1 = counted (cl_count, cl_sample; set by the last kernel of the
  // count, before the write kernels that test it), 2 = plan only (cl_plan);
  // cleared again below if the plan failed
  hipError_t eb = launch_plan_back(dhdr, h, t, s, ev0, ev1);
  if (eb == hipSuccess && mode == 2) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, &dhdr->planned, 2u);
    eb = hipGetLastError();
  }
  if (eb == hipSuccess && into) eb = launch_write(dhdr, t, into->edges, 0, into->cap, into->graph_offsets, s);
  float lane_ms = -1.0f;
  // the header and the edge counts in one read-back
  std::vector<unsigned char> head(F.off_m + 8ull * G);
  if (eb == hipSuccess) {
    eb = hipMemcpyAsync(head.data(), dhdr, head.size(), hipMemcpyDeviceToHost, s);
    if (eb == hipSuccess) eb = hipStreamSynchronize(s);
  }
  if (eb == hipSuccess) {
    memcpy(&back, head.data(), sizeof(back));
    memcpy(m_out, head.data() + F.off_m, 8ull * G);
    if (ev0 && hipEventElapsedTime(&lane_ms, ev0, ev1) != hipSuccess) {
      lane_ms = -1.0f;
      (void)hipGetLastError();   // leave no error behind for the caller's next HIP call
    }
  }
  if (eb != hipSuccess) return CL_ERR_DEVICE;
  if (back.status) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, &dhdr->planned, 0u);
    (void)hipGetLastError();
    return status_error(back.status);
  }
  // the lane kernel's duration, stored by a kernel (no host buffer to keep alive)
  uint32_t ms_bits;
  memcpy(&ms_bits, &lane_ms, sizeof(ms_bits));
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, reinterpret_cast<uint32_t*>(&dhdr->lane_ms), ms_bits);
  CL_TRY(hipGetLastError());
  if (into) {
    uint64_t total = 0;
    for (uint32_t i = 0; i < G; ++i) total += m_out[i];
    if (total > into->cap) return CL_ERR_CAPACITY;
  }
  return CL_OK;
}

cl_status cl_count(const cl_graph* g, uint32_t G, const cl_tuning* t, void* ws, uint64_t ws_bytes, uint64_t* m_out,
                   uint64_t* ws_required, void* stream) {
  return plan_common(g, G, t, ws, ws_bytes, m_out, ws_required, stream, 0u);
}

cl_status cl_sample(const cl_graph* g, uint32_t G, const cl_tuning* t, void* ws, uint64_t ws_bytes, uint64_t* m_out,
                    uint64_t* ws_required, void* stream) {
  return plan_common(g, G, t, ws, ws_bytes, m_out, ws_required, stream, 1u);
}

cl_status cl_sample_into(const cl_graph* g, uint32_t G, const cl_tuning* t, void* ws, uint64_t ws_bytes,
                         uint32_t* edges, uint64_t cap, uint64_t* graph_offsets, uint64_t* m_out,
                         uint64_t* ws_required, void* stream) {
  if (cap > 0 && !edges) return CL_ERR_INVALID_ARG;
  const IntoOut into{edges, cap, graph_offsets};
  return plan_common(g, G, t, ws, ws_bytes, m_out, ws_required, stream, 1u, &into);
}

}  // extern "C"

// ------------------------------------------------ no-allocation variant
// The workspace of cl_sample_into_noalloc: a fixed array in device memory,
// one copy per GPU (allocated when the code object is loaded, held until the
// process ends).  Host code never passes `scratch` itself to a kernel or a
// copy (on the host the name is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns for the current GPU.
static __device__ __align__(256) unsigned char scratch[CL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of the current GPU's scratch array, looked up once per
// device (with that device current) and kept
cl_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return CL_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return CL_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CL_OK;
}
}  // namespace

extern "C" {

cl_status cl_sample_into_noalloc(const cl_graph* g, uint32_t G, const cl_tuning* t, uint32_t* edges, uint64_t cap,
                                 uint64_t* graph_offsets, uint64_t* m_out, uint64_t* ws_required, void* stream) {
  if (cap > 0 && !edges) return CL_ERR_INVALID_ARG;
  void* ws = nullptr;
  const cl_status st = scratch_of_current_device(&ws);
  if (st != CL_OK) return st;
  // a plan that needs more than the array fails with CL_ERR_WORKSPACE before
  // its sizes are laid out (ws_required reports what it would need)
  const IntoOut into{edges, cap, graph_offsets};
  return plan_common(g, G, t, ws, CL_NOALLOC_SCRATCH_BYTES, m_out, ws_required, stream, 1u, &into);
}

cl_status cl_plan(const cl_graph* g, uint32_t G, const cl_tuning* t, void* ws, uint64_t ws_bytes,
                  uint64_t* ws_required, void* stream) {
  if (G == 0 || G > (1u << 24)) return CL_ERR_INVALID_ARG;
  std::vector<uint64_t> m(G);
  return plan_common(g, G, t, ws, ws_bytes, m.data(), ws_required, stream, 2u);
}

cl_status cl_generate(void* ws, const cl_tuning* t, uint32_t* edges, uint64_t edge_begin, uint64_t cap,
                      uint64_t* graph_offsets, void* stream) {
  if (!ws || (cap > 0 && !edges)) return CL_ERR_INVALID_ARG;
  if (edge_begin + cap < edge_begin) return CL_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  WsHeader* dhdr = static_cast<WsHeader*>(ws);
  // G for the offsets kernel: read from the header (the launch covers up to 2^20 tasks)
  CL_TRY(launch_write(dhdr, t, edges, edge_begin, edge_begin + cap, graph_offsets, s));
  return CL_OK;
}

cl_status cl_degrees(void* ws, const cl_tuning* t, uint32_t* deg, uint64_t deg_len, void* stream) {
  if (!ws || !deg) return CL_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  WsHeader* dhdr = static_cast<WsHeader*>(ws);
  WsHeader back{};
  CL_TRY(hipMemcpyAsync(&back, ws, sizeof(back), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  if (back.magic != kWsMagic) return CL_ERR_NOT_PLANNED;
  if (back.status) return status_error(back.status);
  if (!back.planned) return CL_ERR_NOT_PLANNED;
  if (deg_len < back.total_q) return CL_ERR_CAPACITY;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, &dhdr->queue, 0u);
  hipLaunchKernelGGL((k_lanes<3>), dim3(persistent_grid(t)), dim3(kPersistThreads), 0, s, dhdr,
                     static_cast<uint2*>(nullptr), 0ull, 0ull, deg, kNoRows, kNoStats);
  return hip_status(hipGetLastError());
}

cl_status cl_unit_stats(void* ws, const cl_tuning* t, uint64_t* stats, uint64_t stats_len, uint64_t* units_out,
                        void* stream) {
  if (!ws || (!stats && stats_len > 0)) return CL_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  WsHeader* dhdr = static_cast<WsHeader*>(ws);
  WsHeader back{};
  CL_TRY(hipMemcpyAsync(&back, ws, sizeof(back), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  if (back.magic != kWsMagic) return CL_ERR_NOT_PLANNED;
  if (back.status) return status_error(back.status);
  if (!back.planned) return CL_ERR_NOT_PLANNED;
  if (units_out) *units_out = back.total_nl;
  if (stats_len < 4 * back.total_nl) return CL_ERR_CAPACITY;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(4 * back.total_nl, 256, stream_grid_cap())), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long*>(stats), 4 * back.total_nl);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, &dhdr->queue, 0u);
  hipLaunchKernelGGL((k_lanes<0, true>), dim3(persistent_grid(t)), dim3(kPersistThreads), 0, s, dhdr,
                     static_cast<uint2*>(nullptr), 0ull, 0ull, static_cast<uint32_t*>(nullptr), kNoRows,
                     reinterpret_cast<UnitStat*>(stats));
  return hip_status(hipGetLastError());
}

cl_status cl_generate_csr(void* ws, const cl_tuning* t, uint32_t* col, uint64_t cap, uint64_t* row_ptr,
                          uint64_t row_len, void* stream) {
  if (!ws || !row_ptr || (cap > 0 && !col)) return CL_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  WsHeader* dhdr = static_cast<WsHeader*>(ws);
  WsHeader back{};
  CL_TRY(hipMemcpyAsync(&back, ws, sizeof(back), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  if (back.magic != kWsMagic) return CL_ERR_NOT_PLANNED;
  if (back.status) return status_error(back.status);
  if (back.planned != 1) return CL_ERR_NOT_PLANNED;
  if (row_len < back.total_q || cap < back.total_m) return CL_ERR_CAPACITY;
  unsigned long long* rows = reinterpret_cast<unsigned long long*>(row_ptr);
  const uint32_t cus = std::max<uint32_t>(cus_of_current_device(), 1);
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(back.total_q, 256, stream_grid_cap())), dim3(256), 0, s, rows,
                     back.total_q);
  // one-pass plans: the slots; then the replay of overflowed units (one-pass
  // plans) or of every unit (two-pass plans); then the row offsets
  hipLaunchKernelGGL((k_compact<true>), dim3(cus * 16), dim3(256), 0, s, dhdr, reinterpret_cast<uint2*>(col), 0ull,
                     cap, rows);   // also clears the unit queue
  hipLaunchKernelGGL((k_lanes<4>), dim3(persistent_grid(t)), dim3(kPersistThreads), 0, s, dhdr,
                     reinterpret_cast<uint2*>(col), 0ull, cap, static_cast<uint32_t*>(nullptr), rows, kNoStats);
  CL_TRY(hipGetLastError());
  CL_TRY(device_scan<uint64_t>(RowIn{{}, rows, back.total_q}, RowOut{{}, rows}, back.total_q, back.scan_tmp, s));
  return CL_OK;
}

cl_status cl_plan_info(const void* ws, uint64_t* lanes, uint64_t* heavy_segments, uint64_t* edges,
                       uint64_t* candidates, float* lane_kernel_ms, uint32_t* overflow_lanes,
                       uint64_t* slot_words, void* stream) {
  if (!ws) return CL_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  WsHeader back{};
  CL_TRY(hipMemcpyAsync(&back, ws, sizeof(back), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  if (back.magic != kWsMagic) return CL_ERR_NOT_PLANNED;
  if (lanes) *lanes = back.total_nl;
  if (heavy_segments) *heavy_segments = back.total_nh;
  if (edges) *edges = back.total_m;
  if (candidates) *candidates = back.total_cand;
  if (lane_kernel_ms) *lane_kernel_ms = back.lane_ms;
  if (overflow_lanes) *overflow_lanes = back.overflow;
  if (slot_words) *slot_words = back.total_words;
  if (back.status) return status_error(back.status);
  if (!back.planned) return CL_ERR_NOT_PLANNED;
  return CL_OK;
}

cl_status cl_hash_edges(const uint32_t* edges, uint64_t m, uint64_t index_base, uint64_t* acc, void* stream) {
  if (!acc || (m > 0 && !edges)) return CL_ERR_INVALID_ARG;
  if (m == 0) return CL_OK;
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(k_hash, dim3(grid_for(m, 256, stream_grid_cap())), dim3(256), 0, s,
                     reinterpret_cast<const uint2*>(edges), m, index_base, reinterpret_cast<unsigned long long*>(acc));
  return hip_status(hipGetLastError());
}

// ----------------------------------------------------------- batch graph
cl_status cl_batch_capture(const cl_graph* g, uint32_t G, const cl_tuning* t, void* ws, uint32_t* edges,
                           uint64_t cap, uint64_t* graph_offsets, void** graph_exec_out, void* stream) {
  cl_status st = check_graphs(g, G);
  if (st != CL_OK) return st;
  if (!ws || !graph_exec_out || !stream || (cap > 0 && !edges)) return CL_ERR_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  WsHeader* dhdr = static_cast<WsHeader*>(ws);
  WsHeader h{};
  CL_TRY(hipMemcpyAsync(&h, dhdr, sizeof(h), hipMemcpyDeviceToHost, s));
  CL_TRY(hipStreamSynchronize(s));
  // only a counted plan (cl_count, cl_sample): its sizes bound every replay
  if (h.magic != kWsMagic || h.planned != 1 || h.mode == 2 || h.status) return CL_ERR_NOT_PLANNED;
  if (h.G != G) return CL_ERR_INVALID_ARG;
  const FixedLayout F = fixed_layout(g, G);
  if (F.total_q != h.total_q || F.total_r != h.total_r) return CL_ERR_INVALID_ARG;
  hipGraph_t graph = nullptr;
  CL_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_plan_front(dhdr, h, G, s);
  if (e == hipSuccess) e = launch_plan_back(dhdr, h, t, s);
  if (e == hipSuccess) e = launch_write(dhdr, t, edges, 0, cap, graph_offsets, s);
  hipError_t e2 = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return CL_ERR_DEVICE;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return CL_ERR_DEVICE;
  *graph_exec_out = reinterpret_cast<void*>(exec);
  return CL_OK;
}

cl_status cl_batch_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return CL_ERR_INVALID_ARG;
  return hip_status(hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(graph_exec), as_stream(stream)));
}

cl_status cl_batch_destroy(void* graph_exec) {
  if (!graph_exec) return CL_ERR_INVALID_ARG;
  return hip_status(hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(graph_exec)));
}

// ------------------------------------------------------- expected degree
cl_status cl_expected_degree_workspace(uint64_t n, uint64_t* bytes_out) {
  if (!bytes_out) return CL_ERR_INVALID_ARG;
  const uint64_t nt = (n + kEdColsMin - 1) / kEdColsMin;
  const uint64_t nb = (n + 255) / 256;
  // a, thresholds, gw (float n each), two float partial planes (for the
  // narrowest tiles), A, B (double n), T partials
  *bytes_out = 3 * align_up(4 * (n + 1)) + 2 * align_up(4 * nt * n + 4) + 2 * align_up(8 * (n + 1)) +
               align_up(8 * (nb + 1)) + align_up(8);
  return CL_OK;
}

}  // extern "C"

namespace {
struct EdLayout {
  float *a, *thr, *gw, *pA, *pB;
  double *A, *B, *tp, *T;
  uint32_t nt, nb, nrow;
  int R, C;
};

// tile shape of the expected-degree kernels from the tuning (rows per lane,
// columns per tile); false for a shape that has no instantiation
bool ed_shape(const cl_tuning* t, int* R, int* C) {
  *R = (t && t->ed_rows) ? static_cast<int>(t->ed_rows) : kEdRowsDefault;
  *C = (t && t->ed_cols) ? static_cast<int>(t->ed_cols) : kEdColsDefault;
  return (*R == 1 || *R == 2 || *R == 4) && (*C == 512 || *C == 1024 || *C == 2048);
}

EdLayout ed_layout(void* ws, uint64_t n, int R, int C) {
  EdLayout L{};
  char* base = static_cast<char*>(ws);
  const uint64_t ntmax = (n + kEdColsMin - 1) / kEdColsMin;
  const uint64_t nb = (n + 255) / 256;
  uint64_t off = 0;
  L.a = reinterpret_cast<float*>(base + off);
  off += align_up(4 * (n + 1));
  L.thr = reinterpret_cast<float*>(base + off);
  off += align_up(4 * (n + 1));
  L.gw = reinterpret_cast<float*>(base + off);
  off += align_up(4 * (n + 1));
  L.pA = reinterpret_cast<float*>(base + off);
  off += align_up(4 * ntmax * n + 4);
  L.pB = reinterpret_cast<float*>(base + off);
  off += align_up(4 * ntmax * n + 4);
  L.A = reinterpret_cast<double*>(base + off);
  off += align_up(8 * (n + 1));
  L.B = reinterpret_cast<double*>(base + off);
  off += align_up(8 * (n + 1));
  L.tp = reinterpret_cast<double*>(base + off);
  off += align_up(8 * (nb + 1));
  L.T = reinterpret_cast<double*>(base + off);
  L.nt = static_cast<uint32_t>((n + C - 1) / C);
  L.nb = static_cast<uint32_t>(nb);
  L.nrow = static_cast<uint32_t>((n + static_cast<uint64_t>(kEdLanes) * R - 1) / (static_cast<uint64_t>(kEdLanes) * R));
  L.R = R;
  L.C = C;
  return L;
}

template <int R, int C>
void launch_ed_tiles(bool backward, const EdLayout& L, const float* w, uint64_t n, hipStream_t s) {
  const dim3 grid(L.nrow, L.nt);
  if (backward)
    hipLaunchKernelGGL((k_expdeg_bwd_tile<R, C>), grid, dim3(kEdLanes), 0, s, w, L.thr, L.gw, n, L.pA, L.pB);
  else
    hipLaunchKernelGGL((k_expdeg_tile<R, C>), grid, dim3(kEdLanes), 0, s, w, L.a, n, L.pA);
}

template <int R>
void launch_ed_tiles_r(bool backward, const EdLayout& L, const float* w, uint64_t n, hipStream_t s) {
  if (L.C == 512) launch_ed_tiles<R, 512>(backward, L, w, n, s);
  else if (L.C == 1024) launch_ed_tiles<R, 1024>(backward, L, w, n, s);
  else launch_ed_tiles<R, 2048>(backward, L, w, n, s);
}

void launch_ed(bool backward, const EdLayout& L, const float* w, uint64_t n, hipStream_t s) {
  if (L.R == 1) launch_ed_tiles_r<1>(backward, L, w, n, s);
  else if (L.R == 2) launch_ed_tiles_r<2>(backward, L, w, n, s);
  else launch_ed_tiles_r<4>(backward, L, w, n, s);
}
}  // namespace

extern "C" {

cl_status cl_expected_degree(const float* w, uint64_t n, double S, double* d_out, void* ws, uint64_t ws_bytes,
                             const cl_tuning* t, void* stream) {
  if ((n > 0 && (!w || !d_out)) || !finite_pos(S)) return CL_ERR_INVALID_ARG;
  if (n > (1ull << 31)) return CL_ERR_TOO_LARGE;
  int R = 0, C = 0;
  if (!ed_shape(t, &R, &C)) return CL_ERR_INVALID_ARG;
  uint64_t need = 0;
  cl_expected_degree_workspace(n, &need);
  if (!ws || ws_bytes < need) return CL_ERR_WORKSPACE;
  if (n == 0) return CL_OK;
  hipStream_t s = as_stream(stream);
  const EdLayout L = ed_layout(ws, n, R, C);
  hipLaunchKernelGGL(k_rowscale, dim3(L.nb), dim3(256), 0, s, w, n, S, L.a);
  launch_ed(false, L, w, n, s);
  hipLaunchKernelGGL(k_expdeg_rows, dim3(L.nb), dim3(256), 0, s, w, L.a, n, L.nt, L.pA, d_out);
  return hip_status(hipGetLastError());
}

cl_status cl_expected_degree_backward(const float* w, uint64_t n, double S, const double* grad_d, int s_depends_on_w,
                                      float* grad_w, void* ws, uint64_t ws_bytes, const cl_tuning* t, void* stream) {
  if ((n > 0 && (!w || !grad_d || !grad_w)) || !finite_pos(S)) return CL_ERR_INVALID_ARG;
  if (n > (1ull << 31)) return CL_ERR_TOO_LARGE;
  int R = 0, C = 0;
  if (!ed_shape(t, &R, &C)) return CL_ERR_INVALID_ARG;
  uint64_t need = 0;
  cl_expected_degree_workspace(n, &need);
  if (!ws || ws_bytes < need) return CL_ERR_WORKSPACE;
  if (n == 0) return CL_OK;
  hipStream_t s = as_stream(stream);
  const EdLayout L = ed_layout(ws, n, R, C);
  hipLaunchKernelGGL(k_rowscale, dim3(L.nb), dim3(256), 0, s, w, n, S, L.a);
  hipLaunchKernelGGL(k_threshold, dim3(L.nb), dim3(256), 0, s, L.a, n, L.thr);
  hipLaunchKernelGGL(k_gw, dim3(L.nb), dim3(256), 0, s, w, grad_d, n, L.gw);
  launch_ed(true, L, w, n, s);
  hipLaunchKernelGGL(k_expdeg_bwd_rows, dim3(L.nb), dim3(256), 0, s, w, L.a, grad_d, L.gw, n, L.nt, L.pA, L.pB, L.A,
                     L.B, L.tp);
  hipLaunchKernelGGL(k_sum_dbl, dim3(1), dim3(256), 0, s, L.tp, L.nb, L.T);
  hipLaunchKernelGGL(k_expdeg_grad, dim3(L.nb), dim3(256), 0, s, grad_d, L.A, L.B, L.T, s_depends_on_w, n, S,
                     grad_w);
  return hip_status(hipGetLastError());
}

}  // extern "C"
