// Workspace layout of the generator: per-graph descriptors, the quantised
// weight prefix, per-source cost / segment prefixes, the heavy-segment table
// and the lane plan.  Shared by the kernels and the host entry points.
#pragma once
#include <stdint.h>

namespace cl {

constexpr uint32_t kWsMagic = 0x434C5731u;  // "CLW1"
constexpr uint32_t kCostUnit = 16;          // lane-plan cost units per expected candidate
// Graded units: the last 1/kTailShare of a graph's plan cost is cut into units
// kTailDiv times smaller than the lane budget, so that the lanes still busy
// when the work queue runs dry finish soon after one another (a lane takes
// about 0.5 ms for a unit of the default budget).  Graphs of fewer than
// kTailMinUnits units keep uniform units.
constexpr uint64_t kTailShare = 8;
constexpr uint64_t kTailDiv = 4;
constexpr uint64_t kTailMinUnits = 4096;
constexpr uint32_t kLaneGroup = 64;         // lanes per work item (one wavefront)

// status bits raised on the device
enum : uint32_t {
  kStNonfinite = 1u << 0,
  kStNegative = 1u << 1,
  kStUnsorted = 1u << 2,
  kStBadS = 1u << 3,        // S < w_0, or 0 < w_0 < 2^-960
  kStCapacity = 1u << 4,    // a size exceeded the capacity frozen in the workspace
  kStCostOverflow = 1u << 5,
  kStPlan = 1u << 6,        // a work unit's segment range out of order or past the graph (internal error)
};

struct GraphDesc {
  // written by the host
  const double* w;
  uint64_t n;
  double S;
  uint64_t seed;
  uint64_t u_begin, u_end;
  uint64_t q_off;    // first slot of this graph's Q (n + 1 slots)
  uint64_t r_off;    // first slot of this graph's source prefixes (u_end - u_begin + 1 slots)
  uint64_t budget;   // lane budget in cost units
  // written by the device
  double qscale;     // 2^32 / w_0 (0 when w_0 = 0)
  uint64_t Qbase, Qend;          // global prefix values at the graph's first / last Q slot
  uint64_t C0, C1, SB0, SB1, H0, H1;
  uint64_t H;        // heavy sources (a prefix of the range)
  uint64_t NH;       // heavy segments
  uint64_t hs_off;   // first heavy-table entry
  uint64_t L;        // lanes that carry work
  uint64_t Lm, Zm;   // the first Lm units share the cost [0, Zm); the other L - Lm share [Zm, Z)
  double um, ut;     // units per cost unit below / from Zm (lane plan only)
  uint64_t NL;       // lanes incl. padding to a multiple of 64
  uint64_t lane_off; // first lane
  uint64_t m;        // edges
  uint64_t edge_off; // first edge in the batch output
  uint32_t status;
  uint32_t policy;   // host: 0 = units of equal cost, 1 = units of equal source counts,
                     // 2 = round robin (unit i takes segments i, i + L, i + 2L, ...)
  uint32_t graded;   // host: policy 0 with smaller units for the last share of the cost
  uint32_t pad;
};

struct Triple {
  uint64_t c, k, h;  // cost units, segments, heavy sources
};

// one segment of a heavy source: candidates [j, send) of source u, segment k
struct HSeg {
  uint32_t u, k, j, send;
};

// One work unit's record in the statistics pass (cl_unit_stats).
struct UnitStat {
  uint64_t t0, t1;   // wave clock (s_memrealtime, 100 MHz) when the lane took the unit / finished it
  uint32_t cost;     // plan cost of the unit's segments, in cost units (kCostUnit per expected candidate)
  uint32_t visits;   // candidates the unit visited
  uint32_t edges;    // edges it kept
  uint32_t lane;     // the lane that ran it: wavefront index * 64 + lane in the wavefront
};
static_assert(sizeof(UnitStat) == 32, "UnitStat is four 64-bit words");

// Pointers into the workspace; copied into the workspace header so that
// later calls need only the workspace base.
struct WsHeader {
  uint32_t magic;
  uint32_t G;
  uint64_t total_q, total_r;         // Q slots, source slots
  uint64_t cap_nh, cap_nl;           // capacities of the variable part (0 = not laid out)
  uint64_t bytes_fixed, bytes_total;
  GraphDesc* desc;
  uint64_t* Q;        // [total_q]
  uint64_t* C;        // [total_r] exclusive prefix of cost units
  uint64_t* SB;       // [total_r] exclusive prefix of segment counts
  double* A;          // [total_r] a_u = w_u / S per source of the range
  uint64_t* scan_tmp; // scan partials
  uint64_t scan_tmp_elems;
  HSeg* hseg;         // [cap_nh] heavy segments (segment index order)
  uint32_t* lane_seg; // [cap_nl] first segment (graph-relative index) of each lane
  uint32_t* lane_cnt; // [cap_nl]
  uint64_t* lane_pos; // [cap_nl + 1] exclusive prefix of lane_cnt (edge offsets)
  uint64_t* lane_scan_tmp;
  uint64_t* m_dev;    // [G]
  uint32_t* group_graph; // [cap_nl / 64]
  // one-pass mode: every lane writes into its own slot while it counts
  uint64_t* lane_cum;    // [cap_nl + 1] cumulative plan cost at each lane's first segment
  uint64_t* slot_off;    // [cap_nl + 1] exclusive prefix of the slot capacities (words)
  uint64_t* slot_scan_tmp;
  uint32_t* slots;       // [slot_cap] words: v per edge, (mark, u) where the source changes
  uint32_t* lane_words;  // [cap_nl] words each lane needed
  uint64_t slot_cap;     // capacity of slots (words)
  uint32_t mode;         // 0: count then replay; 1: one pass into slots, then compaction
  uint32_t overflow;     // lanes whose edges exceeded their slot (replayed by the write kernel)
  uint32_t slot_margin;  // 0: mu + 8 sqrt(mu) + 24; 1: no margin
  float lane_ms;         // duration of the last count / one-pass lane kernel (HIP events, ms)
  uint64_t total_cost;   // sum of the graphs' plan costs (cost units)
  // device-written totals
  uint64_t total_nh, total_nl, total_m;
  uint64_t total_seg;   // segments of all graphs
  uint64_t total_cand;  // candidates visited by the count pass
  uint64_t total_words; // slot words the one pass needed
  uint32_t status;
  uint32_t queue;
  uint32_t planned;   // 1 after a successful count
  uint32_t pad2;
  double max_cost_check;
  // processing order of the units by position (single-graph plans; cl_tuning
  // unit_order 2, the default for one graph): perm[t] is the unit handed out
  // t-th; null: index order
  uint32_t* perm;          // [cap_nl]
  uint32_t* order_hist;    // [2 kOrderBins] units per bin, then each bin's next free place
  uint16_t* order_keys;    // [cap_nl] each unit's bin
  uint64_t order_blocks;
};

}  // namespace cl
