// Internal declarations of the dfpr library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dfpr.h"

namespace dfpr {

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* last_error();
void clear_error();

struct Status {
  int code = DFPR_OK;
  bool ok() const { return code == DFPR_OK; }
};

#define DFPR_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::dfpr::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                        __FILE__, __LINE__);                                        \
      return (e_ == hipErrorOutOfMemory) ? DFPR_ENOMEM : DFPR_EHIP;                 \
    }                                                                               \
  } while (0)

#define DFPR_TRY(expr)             \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != DFPR_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------- buffers
// Device sub-allocator over one hipMalloc'ed region: best fit over a free list
// with coalescing, 256-byte granules.  alloc/free never call into the HIP
// runtime, so they neither block nor synchronise the device.  Thread-safe.
class Heap {
 public:
  static constexpr size_t kAlign = 256;
  ~Heap();
  int init(size_t bytes);                 // one hipMalloc'ed region, freed with the heap
  void init_at(void* base, size_t bytes);  // a region lent by the caller
  void* alloc(size_t bytes);  // nullptr when no free block is large enough
  void free(void* p);
  size_t capacity() const { return cap_; }
  size_t used();
  size_t peak();
  size_t largest_free();
  char* base() const { return base_; }
  // Record that the taken blocks are exactly `lens` bytes each, packed from
  // offset 0 in this order (after the caller moved their contents there).
  void repack(const std::vector<size_t>& lens);

 private:
  std::mutex mu_;
  char* base_ = nullptr;
  bool owned_ = false;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> taken_;  // offset -> length
};

// A growable device buffer (bytes).  Growth frees and reallocates; contents
// are not preserved.  With a heap the memory comes from it (exact sizes).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Heap* heap = nullptr;
  int ensure(size_t want);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// HIP-event timing of kernel spans.  Events are recorded between launches and
// read only after the caller's final stream synchronisation.
enum TimeTag : int {
  kTPull0 = 0, kTPull1, kTPull2, kTCommit, kTBin, kTMark, kTSort, kTRebuildOut, kTRebuildIn, kTTotal, kTNum
};
struct EventPool {
  std::vector<hipEvent_t> ev;
  struct Span { int tag; size_t a, b; };
  std::vector<Span> spans;
  size_t used = 0;
  bool on = false;
  hipStream_t s = nullptr;
  void reset(bool enable, hipStream_t st) {
    on = enable;
    s = st;
    used = 0;
    spans.clear();
  }
  int record(size_t* idx) {
    if (used == ev.size()) {
      hipEvent_t e;
      DFPR_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
    DFPR_HIP(hipEventRecord(ev[used], s));
    *idx = used++;
    return DFPR_OK;
  }
  // start a span; *tok identifies it for stop()
  int start(size_t* tok) {
    *tok = 0;
    return on ? record(tok) : DFPR_OK;
  }
  int stop(int tag, size_t tok) {
    if (!on) return DFPR_OK;
    size_t b;
    DFPR_TRY(record(&b));
    spans.push_back(Span{tag, tok, b});
    return DFPR_OK;
  }
  // sum the spans per tag (stream must be synchronised)
  int collect(double* ms, int* cnt) {
    for (const Span& sp : spans) {
      float t = 0.f;
      DFPR_HIP(hipEventElapsedTime(&t, ev[sp.a], ev[sp.b]));
      ms[sp.tag] += t;
      cnt[sp.tag] += 1;
    }
    spans.clear();
    used = 0;
    return DFPR_OK;
  }
  void destroy() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }
};

struct Csr {
  int32_t* off = nullptr;  // n+1
  int32_t* idx = nullptr;  // capacity
};

// Reductions that many workgroups feed go to kSlots accumulators, each on its
// own 128-byte line (workgroup b uses slot b % kSlots), and one small kernel
// folds the slots: a single hot address would serialise the atomics of every
// workgroup on the chip.
constexpr int kSlots = 64;
constexpr int kSlotStride = 16;  // 16 x 8 bytes = 128 bytes between slots
constexpr int kBins = DFPR_BINS;
enum AccRow : int {
  kAccEdges0 = 0,          // per-bin in-degree sums of a binning pass (kBins rows)
  kAccEver = kBins,        // vertices processed at least once
  kAccCnt = kBins + 1,     // dense pull: affected vertices
  kAccAffEdges = kBins + 2,// dense pull: summed in-degree of the affected vertices
  kAccXEdges = kBins + 3,  // dense pull: summed out-degree of the expanding vertices
  kAccStayEdges = kBins + 4,  // dense pull: summed in-degree of the kept vertices
  kAccOutEdges = kBins + 5,   // binning pass: summed out-degree of the binned vertices
  kAccCarry = kBins + 6,      // dense pull: unprocessed vertices whose rank was copied over
  kAccRows = kBins + 7
};

// Per-update control block in device memory.  The compact head is read back
// once per iteration; the slot arrays are the spread accumulators.
struct IterCtl {
  unsigned long long dR;     // L-inf change of the last finished pull (double bits)
  int64_t bin_end[kBins];    // worklist end offset of each bin
  int64_t bin_edges[kBins];  // summed in-degree of each bin
  int64_t n_apply[6];        // apply: eff ins, eff del, self dels, eff count, error flag, m_new
  int64_t n_local[6];        // row-local apply: touched rows (out, in), rows without room,
                             // merge work items (out, in)
  int64_t big_count;         // entries in the long out-row list
  int64_t ever_count;        // vertices processed at least once in this update
  int64_t dense_cnt;         // dense pull: affected vertices of the last iteration
  int64_t dense_edges;       // dense pull: their summed in-degree
  int64_t dense_xedges;      // dense pull: summed out-degree of its expanding vertices
  int64_t dense_sedges;      // dense pull: summed in-degree of its kept vertices
  int64_t active;            // member graphs not yet converged (1/0 for a plain graph)
  int64_t bin_out_edges;     // summed out-degree of the vertices of the last binning pass
  int64_t dense_carry;       // dense pull: unprocessed vertices whose rank was copied over
  // single-launch loop outcome: iterations, converged, last L-inf change (bits)
  int64_t fused_iters, fused_converged;
  unsigned long long fused_last;
  int64_t fused_err;  // grid barrier gave up waiting (never expected)
  int64_t pad[1];
  unsigned long long acc_slots[kAccRows][kSlots * kSlotStride];
  // single-launch loop: L-inf change of iteration i in fused_dr[(i % 3) * kSlotStride];
  // batches: members still running after iteration i in fused_act[(i % 3) * kSlotStride]
  unsigned long long fused_dr[3 * kSlotStride];
  unsigned long long fused_act[3 * kSlotStride];
  // grid barrier of the single-launch loop: 32 group counters, a root counter
  // and a generation, each on its own 128-byte line
  unsigned bar_leaf[32 * 32];
  unsigned bar_root[32];
  unsigned bar_gen[32];
};
constexpr size_t kCtlHead = offsetof(IterCtl, pad);

// Work split of the pull kernel's chunked bin and of long out-rows.
constexpr int kPullChunk = 4096;   // in-edges per workgroup work item (bin 5)
constexpr int kMarkChunk = 1024;   // out-edges per workgroup work item
constexpr int kBigRow = 1024;      // out-rows longer than this go to the chunked marking
constexpr int kGSub = 8;           // spread slots per member graph for its L-inf reduction
constexpr int64_t kPartVertices = (int64_t)8 << 20;  // 64 MB of contributions per batch part
// Default single-launch limit of batch handles (arena edges).  Many small
// members gain most from it; on large arenas the launch-per-iteration loop is
// faster (frontier-form iterations, twice the occupancy of the pull).
constexpr int64_t kFusedBatchEdges = (int64_t)1 << 26;

// ---- two-phase dense pull (twophase.hip): blocks of 8192 sources, buckets
// of 4096 destinations, at most kTpMaxB buckets (2^25 vertices)
constexpr int kTpSrcBits = 13, kTpSrc = 1 << kTpSrcBits;
constexpr int kTpDstBits = 12, kTpDst = 1 << kTpDstBits;
constexpr int kTpMaxB = 8192, kTpMaxS = kTpMaxB / 2;
constexpr int64_t kTpItemBuild = 65536;  // in-CSR slots per layout-build work item
constexpr int64_t kTpItem1 = 131072;     // edges per phase-one work item
constexpr int64_t kTpItem2 = 65536;      // edges per phase-two work item
constexpr int kTpFixBits = 96;           // contributions on a grid of 2^-96

// A non-negative double below 2^31 as the integer nearest to x * 2^96
// (ties to even), in two 64-bit words.  Exact for x >= 2^-44.
struct Fix128 {
  uint64_t lo, hi;
};
__device__ __forceinline__ Fix128 fix128(uint64_t bits) {
  Fix128 x{0, 0};
  const int e = (int)(bits >> 52);
  if (e == 0) return x;  // zero or subnormal: far below half a grid step
  const uint64_t mnt = (bits & ((1ull << 52) - 1)) | (1ull << 52);
  const int sh = e - (1075 - kTpFixBits);  // x * 2^96 = mnt * 2^sh
  if (sh >= 64) {
    x.hi = mnt << (sh - 64);
  } else if (sh > 0) {
    x.lo = mnt << sh;
    x.hi = mnt >> (64 - sh);
  } else if (sh == 0) {
    x.lo = mnt;
  } else if (sh > -54) {
    const int t = -sh;
    const uint64_t q = mnt >> t, r = mnt & ((1ull << t) - 1), h = 1ull << (t - 1);
    x.lo = q + (uint64_t)(r > h || (r == h && (q & 1)));
  }
  return x;
}
// hi * 2^-32 + lo * 2^-96 rounded to the nearest double (ties to even): the
// top 64 bits with a sticky bit for the rest, converted once.
__device__ __forceinline__ double unfix128(uint64_t lo, uint64_t hi) {
  if (hi == 0) return (double)lo * 0x1p-96;
  const int z = __clzll((long long)hi);
  const uint64_t top = z ? (hi << z) | (lo >> (64 - z)) : hi;
  const uint64_t rest = z ? lo << z : lo;
  return ldexp((double)(top | (uint64_t)(rest != 0)), -32 - z);
}

struct TwoPhase {
  bool on = false;
  uint64_t built = ~0ull;  // csr_version the layout was built from
  int32_t nS = 0, nB = 0;
  int64_t m = 0;
  int n1 = 0, n2 = 0;  // work items of phase one and two
  DevBuf p1, dstl, val, cnt, tabB, tabS, delta, tmp, glo, ghi, gfl, split, starts, bad, bitems, items1, items2;
  ~TwoPhase();
};

}  // namespace dfpr

struct dfpr_graph {
  std::mutex mu;
  int device = 0;
  bool poisoned = false;
  int32_t n = 0;
  int64_t m = 0;
  int64_t slots = 0;  // entries of each index array, slack included (out.off[n] == in.off[n])
  int32_t slack = 0;  // free slots given to every row at the last re-layout
  int64_t cap = 0;    // edge capacity of each index array
  int id_bits = 1;   // bits per vertex id in packed sort keys
  // members of a batch (disjoint union; member k owns vertices [vbase[k], vbase[k+1]))
  int32_t ngraphs = 1;
  std::vector<int64_t> vbase;        // host, ngraphs + 1
  int32_t* gidv = nullptr;           // n: member of each vertex (null for a plain graph)
  int64_t* vbase_d = nullptr;        // device copy of vbase (batches)
  int32_t* nk = nullptr;             // ngraphs: vertex count of each member
  uint8_t* done = nullptr;           // ngraphs: member converged in this update
  int gsub = 1;                      // spread L-inf slots per member (kSlots for a plain graph)
  unsigned long long* gslots = nullptr;  // ngraphs * gsub spread L-inf slots (kSlotStride apart)
  double* g_dr = nullptr;            // ngraphs: last L-inf change
  int32_t* g_iters = nullptr;        // ngraphs: iterations run
  int64_t* g_ever = nullptr;         // ngraphs: vertices processed at least once
  int64_t* g_eff = nullptr;          // 4 * ngraphs: eff. ins/del pairs, edges after, ignored self dels
  void* g_host = nullptr;            // pinned mirror of g_dr, g_iters, g_ever, g_eff, done
  int32_t* perm = nullptr;  // n: caller id -> internal id (null: identity)
  int32_t* inv = nullptr;   // n: internal id -> caller id
  double* rint = nullptr;   // n: ranks in internal order (when relabelled)
  dfpr::Csr out, in;        // current canonical CSRs
  dfpr::Csr out2, in2;      // rebuild targets (swapped in after a batch)
  // A served graph keeps its CSRs in the server's heap: out and in share one
  // block (csr_block) and the rebuild targets are lent per request.
  dfpr::Heap* csr_heap = nullptr;
  void* csr_block = nullptr;
  // True degrees |out(v)| and |in(v)| (self-loop included).  Row v of a CSR
  // holds its degree's worth of neighbours, ascending, from off[v] on; any
  // further entries up to off[v+1] are free slots holding the pad id n.
  int32_t* out_deg = nullptr;
  int32_t* in_deg = nullptr;
  // rank scratch (n entries each)
  double* contrib = nullptr;   // R[u]/|out(u)| of the current iterate
  double* contrib2 = nullptr;  // ping-pong partner for Static/ND
  double* rn = nullptr;        // ping-pong rank buffer for Static/ND
  uint8_t* flag_cur = nullptr;   // affected in this iteration; between updates:
                                 // pending targets of effective deletions
  uint8_t* flag_next = nullptr;  // affected in the next iteration
  uint8_t* xflag = nullptr;      // expands in this iteration
  uint8_t* xflag2 = nullptr;     // dense mode: expand flags of the previous iteration
  uint8_t* ever = nullptr;       // processed at least once in this update
  uint8_t* pend_src = nullptr;   // pending sources of effective changes
  uint8_t* touched_out = nullptr, *touched_in = nullptr;  // rows changed by the batch
  int32_t* delta_out = nullptr, *delta_in = nullptr;      // row length changes
  int32_t* worklist = nullptr;   // n entries: thread bin | wave bin | block bin
  int32_t* all_bins = nullptr;   // n entries: every vertex, binned per part (Static/ND, dense form)
  // Parts of the vertex range pulled one launch after another.  A batch is cut
  // at member boundaries into parts of about kPartVertices vertices, so each
  // launch gathers from one part's contributions only (they stay in the
  // Infinity Cache); a plain graph is one part.
  struct Part {
    int64_t lo = 0, hi = 0;
    int64_t bin_end[DFPR_BINS] = {0};    // relative to lo
    int64_t bin_edges[DFPR_BINS] = {0};
  };
  std::vector<Part> parts;
  bool all_bins_valid = false;
  bool all_chunks_valid = false;  // all_chunk_pre matches all_bins
  dfpr::IterCtl* ctl = nullptr;      // device
  dfpr::IterCtl* ctl_host = nullptr; // pinned host mirror
  int64_t* scan_tmp = nullptr;       // block sums for scans over n
  size_t scan_tmp_n = 0;
  int64_t* bin_blk = nullptr;        // per-block bin counts (kBins * ceil(n/2048) + 1)
  int64_t* chunk_pre = nullptr;      // n+1: chunk prefix of the chunked bin (frontier worklist)
  int64_t* all_chunk_pre = nullptr;  // n + parts + 1: the same for the all-vertex bins (part k at lo + k)
  int64_t* piece_pre = nullptr;      // n/64+2: CSR rebuild work pieces per 64-row group
  double* partial = nullptr;         // partial sums of pull chunks
  int64_t partial_n = 0;
  int32_t* big_list = nullptr;       // n: vertices with long out-rows to mark
  int64_t* big_pre = nullptr;        // n+1: chunk prefix of big_list
  // growable batch scratch
  dfpr::DevBuf keys_a, keys_b, keys_c, sort_hist, eff_pre, batch_in, keys_in;
  dfpr::DevBuf row_work;  // row-local apply: work-item prefixes of the touched rows
  bool pending_any = false;  // an apply happened since the last DF/DF-P update
  int32_t bounds[5] = {4, 16, 128, 2048, 32768};  // in-degree bin limits (dfpr_set_tuning)
  int32_t* arrive = nullptr;  // n: per-vertex chunk arrival counters of bin 5
  int32_t* partial_x = nullptr;  // per-chunk "an in-neighbour expanded" flags (dense mode)
  bool timing = false;        // record HIP-event timings of every call
  int64_t fused_limit = 1 << 22;  // run whole updates in one launch up to this many edges (0: never);
                                  // batch handles: kFusedBatchEdges by default
  int32_t fused_share = 1;        // a single-launch loop takes 1/fused_share of the device's budget
  void* fused_parts = nullptr;    // device: one pull layout per part for the single-launch loop (batches)
  void* fused_parts_host = nullptr;  // pinned mirror of the part table last copied
  bool fused_parts_stale = true;
  dfpr::EventPool pool;
  uint64_t csr_version = 0;      // bumped whenever the CSRs' contents change
  dfpr::TwoPhase* tp = nullptr;  // two-phase dense pull (dfpr_set_two_phase), null when off
  // vertex-proportional scratch of apply and rank updates, carved from one block
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  bool scratch_owned = false;  // block hipMalloc'ed by the handle (else lent by a server heap)
};

namespace dfpr {

// ---- primitives (prim.hip)
// Exclusive scan of in[0..n) (int64) into out[0..n]; out[n] = total.  tmp needs
// scan_tmp_elems(n) entries.
size_t scan_tmp_elems(int64_t n);
int scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// Row offsets: out[u] = sum_{w<u} (base_off[w+1]-base_off[w] + delta[w]), u in [0,n].
int scan_row_offsets(const int32_t* base_off, const int32_t* delta, int32_t* out, int32_t n,
                     int64_t* tmp, hipStream_t s);
// Stable LSD radix sort of n 64-bit keys on their bits [lo_bit, bits) (keys
// equal there keep their input order).  Result lands in *keys (pointer may be
// swapped with alt).  hist must hold radix_hist_elems(n).
size_t radix_hist_elems(int64_t n);
int radix_sort(uint64_t** keys, uint64_t** alt, int64_t n, int bits, int64_t* hist,
               int64_t* hist_scan_tmp, hipStream_t s, int lo_bit = 0);
size_t radix_scan_tmp_elems(int64_t n);
// Stable compaction: out[k] = in[i] for the i with keep(i); count written to *count_dev.
int compact_keys(const uint64_t* in, const uint8_t* keep, uint64_t* out, int64_t n,
                 int64_t* count_dev, int64_t* tmp_pre, int64_t* tmp, hipStream_t s);

// ---- graph (graph.hip)
int graph_create(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, dfpr_where where,
                 int64_t edge_capacity, int32_t flags, hipStream_t s, dfpr_graph** out,
                 const std::vector<int64_t>* members = nullptr);
int batch_create(int32_t count, const int32_t* n, const int64_t* m, const int32_t* const* src,
                 const int32_t* const* dst, dfpr_where where, int32_t flags, hipStream_t s, dfpr_graph** out);
int batch_apply(dfpr_graph* g, const int64_t* n_del, const int32_t* const* del_src, const int32_t* const* del_dst,
                const int64_t* n_ins, const int32_t* const* ins_src, const int32_t* const* ins_dst, dfpr_where where,
                hipStream_t s, dfpr_batch_info* info);
int graph_destroy(dfpr_graph* g);
// Scratch block: size, attach (carve the arrays, clear the zero-initialised
// prefix on stream s) and detach.  Apply and rank updates need it attached.
size_t scratch_size(const dfpr_graph* g);
int attach_scratch(dfpr_graph* g, void* block, size_t bytes, hipStream_t s);
void detach_scratch(dfpr_graph* g);
// Device bytes an apply of nk batch pairs takes from its growable buffers.
size_t apply_buffer_bytes(int64_t nk, bool host_input);
// One block holding an out-CSR and an in-CSR of n rows and cap edges: its
// size, and the four arrays carved from it.
size_t csr_pair_bytes(int32_t n, int64_t cap);
void carve_csr_pair(void* block, int32_t n, int64_t cap, Csr* out, Csr* in);
// Served graphs: move the CSRs into one block of `heap` (the rebuild targets
// are released; requests lend them), or make room for cap edges in the chunk
// partial sums before a request whose insertions raise the capacity.
int move_csrs_to_heap(dfpr_graph* g, Heap* heap, hipStream_t s);
int ensure_partials(dfpr_graph* g, int64_t cap);
int graph_export(const dfpr_graph* g, int in_csr, int32_t* off, int32_t* idx, dfpr_where where,
                 hipStream_t s);
int graph_apply(dfpr_graph* g, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where,
                hipStream_t s, dfpr_batch_info* info);
// Re-lay out both CSRs with `slack` free slots per row (Section 3.2 batches
// then merge into rows that have room, without moving the others).
constexpr int32_t kMaxRowSlack = 1 << 16;
int graph_set_row_slack(dfpr_graph* g, int32_t slack, hipStream_t s);
// two-phase dense pull (twophase.hip)
bool tp_supported(const dfpr_graph* g, const char** why);
int tp_build(dfpr_graph* g, hipStream_t s);
int tp_phases(dfpr_graph* g, const double* contrib, const uint8_t* xflag, hipStream_t s);
// Slots an apply of n_ins insertions may need in each index array.
int64_t slots_bound(const dfpr_graph* g, int64_t n_ins);
// graph_apply with its sort and staging buffers in the library's fixed device
// scratch (no device allocation): at most DFPR_NOALLOC_MAX_PAIRS pairs and no
// growth of the edge capacity.
int graph_apply_noalloc(dfpr_graph* g, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                        int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where,
                        hipStream_t s, dfpr_batch_info* info);

// ---- serving form (server.hip)
int server_create(size_t heap_bytes, int32_t lanes, dfpr_mode mode, const dfpr_params& p, dfpr_server** out);
int server_destroy(dfpr_server* sv);
int server_add_graph(dfpr_server* sv, dfpr_graph* g, const double* r0, int32_t* gid);
int server_submit(dfpr_server* sv, int32_t gid, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                  int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, double* r_out, int64_t* ticket);
int server_wait(dfpr_server* sv, int64_t ticket, dfpr_stats* st, dfpr_batch_info* info, double* latency_ms,
                double* queue_ms);
int server_ranks(dfpr_server* sv, int32_t gid, double* r_out, dfpr_where where);
int server_stats(dfpr_server* sv, dfpr_server_stats* out);
int32_t server_graph_n(dfpr_server* sv, int32_t gid);
int server_set_active_lanes(dfpr_server* sv, int32_t k);

// ---- ranks (rank.hip)
int update_ranks(dfpr_graph* g, dfpr_mode mode, const dfpr_params& p, const double* r_prev,
                 double* r_out, hipStream_t s, dfpr_stats* st, dfpr_stats* per_member = nullptr);
int autotune(dfpr_graph* g, hipStream_t s, int32_t* bounds_out, double* ms_out);

inline int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) b++;
  return b;
}

inline unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (int64_t)cap) g = cap;
  return (unsigned)g;
}

}  // namespace dfpr

// ---------------------------------------------------------------- device helpers
namespace dfpr {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
  return x;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// lower_bound over a sorted int32 range
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t* a, int32_t lo, int32_t hi, int32_t x) {
  while (lo < hi) {
    int32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* a, int64_t lo, int64_t hi, uint64_t x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace dfpr
