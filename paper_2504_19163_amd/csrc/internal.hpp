// Library-internal state of a bound hierarchy and the launch entry points of
// the kernels (one translation unit per stage).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/bbc.h"
#include "geom_dev.hpp"

namespace bbc {

// Subdivision queue item: tuple id and the box index at the item's depth,
// packed as iu << 14 | iv (depth <= 14).
struct QItem {
  uint32_t tuple;
  uint32_t code;
};

constexpr int kCodeBits = 14;
constexpr int kMaxDepth = 14;

// One request of a batched query launch: sampling parameters and where its
// points start inside the batch.
struct ReqDesc {
  float W;
  uint32_t pad;
  uint64_t seed;
  int64_t base;   // point index of the request's first point (Philox counter)
  int64_t start;  // offset of the request's first point inside the batch
};

// Device counters of one build (zeroed by a fill kernel at the start).
struct BuildCounters {
  uint32_t n_init;                 // unsettled tuples queued for domain initialisation
  uint32_t n_l0_fp64;              // level-0 boxes queued for FP64 re-evaluation
  uint32_t n_leaves;
  uint32_t n_boxes;
  uint32_t n_fp64;
  uint32_t n_live;                 // tuples with a root box
  uint32_t overflow;               // bit flags: 1 queue, 2 leaves, 4 grid entries, 8 fp64 queue, 16 init,
                                   // 32 subdivision records
  uint32_t max_depth;
  uint32_t n_triples;              // grid entries wanted when they overflowed the capacity
  uint32_t n_entries;              // (cell, tuple) entries of the grid
  uint32_t n_inf;
  uint32_t n_cover;                // tuples in the cover-all list
  uint32_t qcount[kMaxDepth + 2];  // items at each depth
  uint32_t fcount[kMaxDepth + 2];  // FP64 items at each depth
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Work space of one staged query launch, carved from one allocation (a
// handle's own buffer or a serving batch's region of the arena).
struct StagedWork {
  uint32_t* cell = nullptr;
  float* gamma = nullptr;
  uint32_t* cnt = nullptr;
  uint32_t* off = nullptr;
  double2* tgt = nullptr;  // receiver coordinates (u, v) of each point
  uint32_t* redo = nullptr;  // pairs left to the redo kernel
  void* scan = nullptr;
  uint32_t* pair_pt = nullptr;
  uint32_t* pair_t = nullptr;
  float* pair_p = nullptr;
  double* pair_c = nullptr;
  uint8_t* pair_nr = nullptr;
  size_t pts = 0, pairs = 0;  // capacities
};

// Launch-shape knobs (bbc_set_tuning; tuning.json written by the package's autotuner).
struct Tuning {
  int query_waves = 2;        // fused query: minimum waves per SIMD (register budget 256 / 128)
  int query_grid = 256 * 64;  // fused query: persistent workgroups
  int query_tile = 16;        // fused query: shading points per wave (16, 32 or 64)
  int timing = 0;             // record events around the query's dominant kernel
  int build_grid_per_cu = 0;  // persistent build kernels: workgroups per CU (0: one resident round)
  int newton_steps = 4;       // staged query: FP32 iterations per pooled Newton pass (0: lane per pair)
  int newton_results = 96;    // pooled Newton: accepted roots kept per 64 pairs before pairs are redone
  int64_t staged_pairs = int64_t(1) << 28;  // worst-case pairs of one staged launch (slices a larger query)
  int graph = 0;              // staged query: 1 = replay the launches as a HIP graph
  int rr_outlined = 0;        // two-reflection subdivision: box evaluation as a called function
  int newton_grid_per_cu = 0; // pooled Newton workgroups per CU (0: occupancy API)
  int build_graph = 0;        // build: 1 = replay the launch sequence as a HIP graph
  int subdiv_split = 1;       // reflection subdivision from split polynomials: 0 off, 1 on, n > 1 on with room for n records at first
};

// A staged query's launches captured into a HIP graph on a stream of the
// library's own, and the executable graph updated in place for each call.
struct QueryGraph {
  hipStream_t stream = nullptr;  // capture and replay stream (non-blocking, default priority)
  hipEvent_t in = nullptr, out = nullptr;  // orders the replay after / before the caller's stream
  hipGraphExec_t exec = nullptr;
  int64_t launches = 0, instantiations = 0;
};
void release_graph(QueryGraph& g);
// Capture the launches that `enqueue(cs)` makes on stream cs into a graph and
// update the executable graph *exec with it (instantiated when absent or when
// the update is refused).
template <class F>
bbc_status capture_into(hipStream_t cs, hipGraphExec_t* exec, int64_t* instantiations, F&& enqueue);
// capture_into on g's stream, then replay g's executable graph there, ordered
// after the work already on `caller` and before the caller's later work.
template <class F>
bbc_status run_as_graph(QueryGraph& g, hipStream_t caller, F&& enqueue);

struct Bounds {
  int device = 0;
  Tuning tune;
  bbc_subdiv_params params{};
  DevScene scene{};       // device pointers into the buffers below
  int64_t n_tuples = 0;   // tuples the build works on (constructed pairs for two reflections)
  int64_t n_dense = 0;    // emitters x triangles (x second-surface triangles)
  int64_t tuples_cap = 0;
  int rec_floats = kRecFloats;
  // scene copies
  DevBuf pos, nrm, epos, eI, pos2, nrm2, eedge;
  // tuple construction (two reflections): second-surface boxes, per-row counts
  // and offsets, pair numbers
  DevBuf box2, rowcount, rowoff, tid;
  // build work space
  DevBuf counters;        // BuildCounters
  DevBuf root;            // float4 [n_tuples]
  DevBuf init_q;          // uint32 [n_tuples]
  DevBuf l0f_q;           // uint32 [n_tuples]
  DevBuf q[2];            // QItem ping-pong
  DevBuf fq;              // QItem FP64 queue
  size_t q_cap = 0, fq_cap = 0;
  // leaves (unsorted, then grouped by tuple)
  DevBuf lt, lc, lu, le;      // tuple u32, code u32, ukbox float4, E float2
  DevBuf gl_t, gl_c, gl_u, gl_e;  // grouped by tuple
  DevBuf st, sc, su, se;      // grouped by tuple, ordered by code
  DevBuf sug;                 // union of the receiver bounds of each run of kLeafGroup sorted leaves
  size_t leaf_cap = 0;
  DevBuf tcount, toff, tcur;  // per-tuple counts / offsets [n_tuples + 1] / cursors
  // receiver grid
  DevBuf lrect;               // cell rectangle, tuple and E_hi of each sorted leaf
  DevBuf lcoarse;             // the rectangle in tiles of 16 cells (padded by two scan steps)
  size_t grid_cap = 0;        // capacity of the grid entry arrays gt / ge
  DevBuf ccount, coff;        // per-cell counts / offsets [G*G + 2]: the last slice is the cover-all list
  DevBuf gt, ge;              // entries: tuple u32, E~ float, sorted by tuple per cell
  DevBuf cflag, cpos, cE;     // cover-all decision per tuple, its slot (scan), largest E_hi
  DevBuf scan_tmp;
  DevBuf trec;                // packed per-tuple records for the query [n_tuples][32] float
  DevBuf red_tab;             // degree-reduction table of the two-reflection irradiance bound
  DevBuf srec[2];             // reflection subdivision: children's polynomial records, by depth parity
  uint32_t srec_cap = 0;      // records per depth parity (0: not sized yet); grown when a depth needs more
  bool red_ready = false;
  // host copies of the final counts
  BuildCounters host{};
  int64_t n_leaves = 0, n_entries = 0, max_cell = 0;
  int64_t device_bytes = 0;
  // query work space (staged form), one allocation grown on demand
  DevBuf qw_buf;
  StagedWork qw;
  DevBuf max_cell_dev;
  DevBuf qcounters;           // 8 x u64 query work counters (filled when host stats are requested)
  // event pairs around the dominant kernel of each launch of the last query
  // (one pair for the fused form, one per slice for the staged form)
  std::vector<hipEvent_t> tev;
  int tev_used = 0;
  // events around the subdivision launches of the last build (timing on)
  hipEvent_t bev[2] = {nullptr, nullptr};
  bool bev_recorded = false;
  int subdiv_launches = 0;
  QueryGraph qgraph;          // the staged query as a graph (BBC_TUNE_GRAPH)
  QueryGraph bgraph;          // the build's launch sequence as a graph (BBC_TUNE_BUILD_GRAPH)
};

// error plumbing
void set_error(const std::string& msg);
bbc_status hip_fail(hipError_t e, const char* what);
#define BBC_HIP(call)                                         \
  do {                                                        \
    hipError_t _e = (call);                                   \
    if (_e != hipSuccess) return ::bbc::hip_fail(_e, #call);  \
  } while (0)

bbc_status ensure(DevBuf& b, size_t bytes, Bounds* owner);
void release(DevBuf& b);

// stage launchers (stream-ordered, no host synchronisation)
bbc_status launch_build(Bounds* b, hipStream_t s);
bbc_status launch_record(Bounds* b, hipStream_t s);
// Sorted leaves in runs of kLeafGroup (leaf i in run i / kLeafGroup, runs may
// span tuples): sug[g] is the union of the receiver bounds of run g, which
// lets the query test a run before its leaves.  n_leaves is read from the
// build counters when `counters` is given, else taken from `n_host`.
constexpr uint32_t kLeafGroup = 8;
bbc_status launch_leaf_groups(Bounds* b, const BuildCounters* counters, uint32_t n_host, hipStream_t s);
bbc_status launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
bbc_status launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
bbc_status launch_pairs(const DevScene& sc, double* box2, uint32_t* rowcount, const uint32_t* rowoff, uint32_t* tid,
                        bool fill, hipStream_t s);
bbc_status launch_query(const Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed, int64_t base,
                        int32_t mode, float* out, float* stats, unsigned long long* counters, hipStream_t s);
bbc_status launch_query_staged(Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed, int64_t base,
                               int32_t mode, float* out, float* stats, unsigned long long* counters, hipStream_t s);
// The staged query over caller-provided work space of `bytes` bytes at `work`
// (device memory, 256-byte aligned): the points run in consecutive slices of
// as many points as the space holds at the worst case.  EBUDGET when one
// point's worst case does not fit.  Allocates nothing.
bbc_status launch_query_staged_in(const Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed,
                                  int64_t base, int32_t mode, float* out, float* stats, void* work, size_t bytes,
                                  hipStream_t s);

// Staged work space: worst-case pair count of n points (every entry of the
// fullest cell selected), bytes for n points and that many pairs, and the
// carving of one allocation of that size.  Pair offsets and pair indices are
// 32-bit, so one staged launch is sized for at most kMaxStagedPairs pairs;
// a larger query runs as consecutive launches over slices of its points.
constexpr size_t kMaxStagedPairs = size_t(1) << 28;
size_t staged_pairs(const Bounds* b, int64_t n);
// Points of one staged launch for a query of n points (at most n).
int64_t staged_slice(const Bounds* b, int64_t n);
size_t staged_bytes(int64_t n, size_t pairs);
void staged_carve(void* base, int64_t n, size_t pairs, StagedWork& w);
// Staged launch over a batch of requests: point i belongs to reqs[preq[i]].
// The batch runs in consecutive slices of staged_slice(b, n) points over the
// work space w, which must hold one slice.  Events (nullable) bracket the
// Newton kernel of the first slice.
bbc_status launch_query_batch(const Bounds* b, const float* pts, int64_t n, const uint16_t* preq,
                              const ReqDesc* reqs, int32_t mode, float* out, const StagedWork& w, hipEvent_t ev0,
                              hipEvent_t ev1, hipStream_t s);

template <class F>
bbc_status capture_into(hipStream_t cs, hipGraphExec_t* exec, int64_t* instantiations, F&& enqueue) {
  BBC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const bbc_status e = enqueue(cs);
  hipGraph_t graph = nullptr;
  const hipError_t he = hipStreamEndCapture(cs, &graph);
  if (e || he != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return e ? e : hip_fail(he, "hipStreamEndCapture");
  }
  if (*exec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult r = hipGraphExecUpdateSuccess;
    if (hipGraphExecUpdate(*exec, graph, &bad, &r) != hipSuccess || r != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(*exec);
      *exec = nullptr;
    }
  }
  hipError_t ie = hipSuccess;
  if (!*exec) {
    ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    ++*instantiations;
  }
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    *exec = nullptr;
    return hip_fail(ie, "hipGraphInstantiate");
  }
  return BBC_OK;
}

template <class F>
bbc_status run_as_graph(QueryGraph& g, hipStream_t caller, F&& enqueue) {
  if (!g.stream) {
    BBC_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
    BBC_HIP(hipEventCreateWithFlags(&g.in, hipEventDisableTiming));
    BBC_HIP(hipEventCreateWithFlags(&g.out, hipEventDisableTiming));
  }
  bbc_status e = capture_into(g.stream, &g.exec, &g.instantiations, enqueue);
  if (e) return e;
  BBC_HIP(hipEventRecord(g.in, caller));
  BBC_HIP(hipStreamWaitEvent(g.stream, g.in, 0));
  BBC_HIP(hipGraphLaunch(g.exec, g.stream));
  BBC_HIP(hipEventRecord(g.out, g.stream));
  BBC_HIP(hipStreamWaitEvent(caller, g.out, 0));
  ++g.launches;
  return BBC_OK;
}

}  // namespace bbc
