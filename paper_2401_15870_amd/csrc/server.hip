// Serving form: a request loop over graphs resident in HBM.
//
// A request applies one batch to one resident graph and updates that graph's
// resident ranks with DF-P (Algorithm 1 from the ranks left by the previous
// request).  Requests for the same graph run one at a time in submission order
// (one writer per graph, Section 3.2); requests for different graphs run
// concurrently on the server's lanes, one HIP stream each, so their kernels
// overlap on the device.  A request is admitted when a lane is free, its graph
// is idle and its scratch (the vertex arrays of the update plus the batch sort
// buffers) fits in what is left of the scratch heap; requests that do not fit
// wait in the queue.  Scratch comes from a device sub-allocator over one region
// reserved at create, so admission and release never call hipMalloc/hipFree.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "dfpr_impl.hpp"

namespace dfpr {

// ---------------------------------------------------------------- heap
Heap::~Heap() {
  if (base_ && owned_) (void)hipFree(base_);
}

void Heap::init_at(void* base, size_t bytes) {
  base_ = static_cast<char*>(base);
  owned_ = false;
  cap_ = bytes / kAlign * kAlign;
  used_ = peak_ = 0;
  free_.clear();
  taken_.clear();
  if (cap_) free_[0] = cap_;
}

int Heap::init(size_t bytes) {
  bytes = (bytes + kAlign - 1) / kAlign * kAlign;
  if (bytes == 0) {
    set_error("heap size must be > 0");
    return DFPR_EINVAL;
  }
  if (hipMalloc((void**)&base_, bytes) != hipSuccess) {
    (void)hipGetLastError();
    base_ = nullptr;
    set_error("device allocation of a %zu-byte scratch heap failed", bytes);
    return DFPR_ENOMEM;
  }
  owned_ = true;
  cap_ = bytes;
  free_[0] = bytes;
  return DFPR_OK;
}

void* Heap::alloc(size_t bytes) {
  bytes = std::max<size_t>(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
  std::lock_guard<std::mutex> lk(mu_);
  auto best = free_.end();
  for (auto it = free_.begin(); it != free_.end(); ++it)  // best fit
    if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
  if (best == free_.end()) return nullptr;
  const size_t off = best->first, len = best->second;
  free_.erase(best);
  if (len > bytes) free_[off + bytes] = len - bytes;
  taken_[off] = bytes;
  used_ += bytes;
  peak_ = std::max(peak_, used_);
  return base_ + off;
}

void Heap::free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  const size_t off = (size_t)(static_cast<char*>(p) - base_);
  auto t = taken_.find(off);
  if (t == taken_.end()) return;
  size_t start = off, len = t->second;
  used_ -= len;
  taken_.erase(t);
  auto next = free_.lower_bound(start);
  if (next != free_.end() && next->first == start + len) {  // merge with the following block
    len += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {  // merge with the preceding block
    auto prev = std::prev(next);
    if (prev->first + prev->second == start) {
      start = prev->first;
      len += prev->second;
      free_.erase(prev);
    }
  }
  free_[start] = len;
}

size_t Heap::used() {
  std::lock_guard<std::mutex> lk(mu_);
  return used_;
}
size_t Heap::peak() {
  std::lock_guard<std::mutex> lk(mu_);
  return peak_;
}
void Heap::repack(const std::vector<size_t>& lens) {
  std::lock_guard<std::mutex> lk(mu_);
  free_.clear();
  taken_.clear();
  size_t off = 0;
  for (size_t len : lens) {
    taken_[off] = len;
    off += len;
  }
  used_ = off;
  if (off < cap_) free_[off] = cap_ - off;
}
size_t Heap::largest_free() {
  std::lock_guard<std::mutex> lk(mu_);
  size_t m = 0;
  for (auto& f : free_) m = std::max(m, f.second);
  return m;
}

}  // namespace dfpr

using namespace dfpr;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  int64_t ticket = 0;
  int32_t gid = 0;
  std::vector<int32_t> ds, dd, is, id;  // host copy of the batch
  double* r_out = nullptr;              // caller's host array (nullable)
  size_t apply_bytes = 0;               // batch sort buffers of this request
  void* scratch = nullptr;              // vertex scratch, taken from the heap at admission
  void* apply_block = nullptr;          // sort buffers, taken from the heap at admission
  void* targets = nullptr;              // rebuild targets (both CSRs), taken from the heap at admission;
                                        // they hold the graph after the apply
  int64_t target_cap = 0;               // their edge capacity
  int rc = DFPR_OK;
  std::string err;
  bool done = false;
  dfpr_stats st{};
  dfpr_batch_info info{};
  Clock::time_point t_submit, t_start, t_done;
};

struct Resident {
  dfpr_graph* g = nullptr;
  double* R = nullptr;      // resident ranks, caller order
  size_t scratch = 0;       // bytes of the graph's vertex scratch block
  bool busy = false;
};

}  // namespace

struct dfpr_server {
  int device = 0;
  dfpr_mode mode = DFPR_DFP;
  dfpr_params params{};
  Heap heap;
  std::deque<Resident> graphs;  // references stay valid while graphs are added
  std::deque<Request*> queue;
  std::unordered_map<int64_t, std::unique_ptr<Request>> requests;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::thread> lanes;
  std::vector<hipStream_t> streams;
  hipStream_t ctl_stream = nullptr;  // add_graph's initial Static solves
  bool stopping = false;
  int64_t next_ticket = 1;
  int32_t in_flight = 0;
  int32_t active_lanes = 0;  // lanes at or above this index take no new work
  dfpr_server_stats counters{};
};

namespace {

// Next admissible request, with its scratch already taken from the heap: scan
// in submission order and skip requests whose graph is busy; a request whose
// scratch does not fit stops the scan (later requests do not overtake it).
// When nothing is in flight and it still does not fit, it never will: it is
// returned with its blocks unset and fails with ENOMEM.
// Idle server (no request in flight, so the only taken blocks are the graphs'
// CSR blocks): slide every CSR block down to the lowest free address, in
// address order, so that the free space is one range.  A block moves to a
// lower address by chunks no longer than the distance it moves, so no chunk's
// source overlaps its destination.  Returns false if a device copy failed.
bool compact(dfpr_server* sv) {
  std::vector<Resident*> res;
  for (auto& r : sv->graphs) res.push_back(&r);
  std::sort(res.begin(), res.end(), [](const Resident* a, const Resident* b) { return a->g->csr_block < b->g->csr_block; });
  hipStream_t s = sv->ctl_stream;
  std::vector<size_t> lens;
  char* cursor = sv->heap.base();
  for (Resident* r : res) {
    dfpr_graph* g = r->g;
    const size_t len = (csr_pair_bytes(g->n, g->cap) + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign;
    char* src = static_cast<char*>(g->csr_block);
    if (src != cursor) {
      const size_t step = (size_t)(src - cursor);
      for (size_t done = 0; done < len; done += step)
        if (hipMemcpyAsync(cursor + done, src + done, std::min(step, len - done), hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
          return false;
      g->csr_block = cursor;
      carve_csr_pair(cursor, g->n, g->cap, &g->out, &g->in);
    }
    lens.push_back(len);
    cursor += len;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  sv->heap.repack(lens);
  return true;
}

// Its blocks: the vertex scratch, the batch sort buffers and the rebuild
// targets, sized for the graph's edges plus the batch's insertions.
Request* pick(dfpr_server* sv) {
  for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
    Request* q = *it;
    Resident& r = sv->graphs[q->gid];
    if (r.busy) continue;
    const dfpr_graph* g = r.g;  // idle: no request changes it meanwhile
    const int64_t need = slots_bound(g, (int64_t)q->is.size());
    q->target_cap = need <= g->cap ? g->cap : std::min<int64_t>(need + need / 4, INT32_MAX);
    for (int attempt = 0; attempt < 2; attempt++) {
      q->scratch = sv->heap.alloc(r.scratch);
      q->apply_block = q->scratch ? sv->heap.alloc(q->apply_bytes) : nullptr;
      q->targets = q->apply_block ? sv->heap.alloc(csr_pair_bytes(g->n, q->target_cap)) : nullptr;
      if (q->targets) break;
      sv->heap.free(q->apply_block);
      sv->heap.free(q->scratch);
      q->scratch = q->apply_block = nullptr;
      if (sv->in_flight > 0) return nullptr;  // wait for running requests to free their blocks
      // nothing runs: the free space is all there will be; gather it in one
      // range (the heap fragments as requests' targets replace CSR blocks)
      // and try once more
      if (attempt == 0 && !compact(sv)) break;
    }
    sv->queue.erase(it);
    return q;
  }
  return nullptr;
}

const std::initializer_list<DevBuf dfpr_graph::*> kApplyBufs = {
    &dfpr_graph::keys_a, &dfpr_graph::keys_b, &dfpr_graph::keys_c, &dfpr_graph::sort_hist,
    &dfpr_graph::eff_pre, &dfpr_graph::batch_in, &dfpr_graph::keys_in, &dfpr_graph::row_work};

int serve(dfpr_server* sv, Request* q, hipStream_t s) {
  Resident& r = sv->graphs[q->gid];
  dfpr_graph* g = r.g;
  if (!q->scratch) {
    set_error("request scratch (%zu + %zu bytes) exceeds the scratch heap (%zu bytes)", r.scratch, q->apply_bytes,
              sv->heap.capacity());
    return DFPR_ENOMEM;
  }
  std::lock_guard<std::mutex> glk(g->mu);
  Heap sub;  // the request's sort buffers come from its own block
  sub.init_at(q->apply_block, q->apply_bytes);
  for (auto b : kApplyBufs) (g->*b).heap = &sub;
  int rc = attach_scratch(g, q->scratch, r.scratch, s);
  // the CSRs are rebuilt into the request's target block, which then holds
  // the graph; the block of the old CSRs goes back to the heap
  const int32_t* old_off = g->out.off;
  const int64_t old_cap = g->cap;
  carve_csr_pair(q->targets, g->n, q->target_cap, &g->out2, &g->in2);
  if (rc == DFPR_OK && q->target_cap > g->cap) {
    rc = ensure_partials(g, q->target_cap);
    g->cap = q->target_cap;
  }
  g->fused_share = sv->active_lanes;  // single-launch loops share the device between lanes
  if (rc == DFPR_OK)
    rc = graph_apply(g, (int64_t)q->ds.size(), q->ds.data(), q->dd.data(), (int64_t)q->is.size(), q->is.data(),
                     q->id.data(), DFPR_HOST, s, &q->info);
  if (g->out.off != old_off) {  // swapped in (a finished apply always swaps)
    (void)hipStreamSynchronize(s);  // nothing reads the old block any more
    sv->heap.free(g->csr_block);
    g->csr_block = q->targets;
    q->targets = nullptr;
  } else {
    g->cap = old_cap;
  }
  g->out2 = g->in2 = Csr();
  if (rc == DFPR_OK) rc = update_ranks(g, sv->mode, sv->params, r.R, r.R, s, &q->st);
  if (rc == DFPR_OK && q->r_out) {
    if (hipMemcpyAsync(q->r_out, r.R, (size_t)g->n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("copy of the result ranks failed");
      rc = DFPR_EHIP;
    }
  }
  (void)hipStreamSynchronize(s);  // nothing of this request may still run when its scratch is returned
  for (auto b : kApplyBufs) {
    (g->*b).release();
    (g->*b).heap = nullptr;
  }
  detach_scratch(g);
  if (rc == DFPR_EHIP) g->poisoned = true;
  return rc;
}

void lane_main(dfpr_server* sv, int lane) {
  (void)hipSetDevice(sv->device);
  hipStream_t s = sv->streams[lane];
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    Request* q = nullptr;
    sv->cv_work.wait(lk, [&] { return sv->stopping || (lane < sv->active_lanes && (q = pick(sv)) != nullptr); });
    if (!q) return;  // stopping with nothing admissible
    Resident& r = sv->graphs[q->gid];
    r.busy = true;
    sv->in_flight++;
    sv->counters.peak_in_flight = std::max<int64_t>(sv->counters.peak_in_flight, sv->in_flight);
    q->t_start = Clock::now();
    lk.unlock();
    clear_error();
    int rc = r.g->poisoned ? (int)DFPR_ESTATE : serve(sv, q, s);
    std::string msg = rc == DFPR_OK ? std::string() : std::string(last_error());
    lk.lock();
    q->rc = rc;
    q->err = msg;
    q->t_done = Clock::now();
    q->done = true;
    sv->heap.free(q->apply_block);
    sv->heap.free(q->scratch);
    sv->heap.free(q->targets);  // unless the graph took them
    q->apply_block = q->scratch = q->targets = nullptr;
    r.busy = false;
    sv->in_flight--;
    sv->counters.completed++;
    if (rc != DFPR_OK) sv->counters.failed++;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

}  // namespace

namespace dfpr {

int server_create(size_t heap_bytes, int32_t lanes, dfpr_mode mode, const dfpr_params& p, dfpr_server** out) {
  std::unique_ptr<dfpr_server> sv(new dfpr_server());
  DFPR_HIP(hipGetDevice(&sv->device));
  sv->mode = mode;
  sv->params = p;
  DFPR_TRY(sv->heap.init(heap_bytes));
  for (int32_t i = 0; i < lanes; i++) {
    hipStream_t s;
    DFPR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    sv->streams.push_back(s);
  }
  DFPR_HIP(hipStreamCreateWithFlags(&sv->ctl_stream, hipStreamNonBlocking));
  sv->active_lanes = lanes;
  for (int32_t i = 0; i < lanes; i++) sv->lanes.emplace_back(lane_main, sv.get(), i);
  *out = sv.release();
  return DFPR_OK;
}

int server_destroy(dfpr_server* sv) {
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->queue.empty() && sv->in_flight == 0; });  // drain
    sv->stopping = true;
    sv->cv_work.notify_all();
  }
  for (auto& t : sv->lanes) t.join();
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  if (sv->ctl_stream) (void)hipStreamDestroy(sv->ctl_stream);
  for (auto& r : sv->graphs) {
    if (r.R) (void)hipFree(r.R);
    if (r.g) graph_destroy(r.g);
  }
  delete sv;
  return DFPR_OK;
}

int server_add_graph(dfpr_server* sv, dfpr_graph* g, const double* r0, int32_t* gid) {
  if (g->ngraphs != 1) {
    set_error("a batch handle cannot be served; add its members as separate graphs");
    return DFPR_EINVAL;
  }
  double* R = nullptr;
  if (hipMalloc((void**)&R, (size_t)g->n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of the resident ranks failed");
    return DFPR_ENOMEM;
  }
  hipStream_t s = sv->ctl_stream;
  const size_t sbytes = scratch_size(g);
  int rc = DFPR_OK;
  {
    std::lock_guard<std::mutex> glk(g->mu);
    if (r0) {
      if (hipMemcpyAsync(R, r0, (size_t)g->n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = DFPR_EHIP;
    } else {
      rc = update_ranks(g, DFPR_STATIC, sv->params, nullptr, R, s, nullptr);  // with the handle's own scratch
    }
    if (rc == DFPR_OK && hipStreamSynchronize(s) != hipSuccess) {
      set_error("resident rank initialisation failed");
      rc = DFPR_EHIP;
    }
    // from now on the CSRs live in the heap and every request borrows its
    // rebuild targets, vertex scratch and sort buffers from it
    if (rc == DFPR_OK) {
      std::lock_guard<std::mutex> lk(sv->mu);  // the heap's layout changes only under the server lock
      rc = move_csrs_to_heap(g, &sv->heap, s);
    }
    if (rc == DFPR_OK) {
      if (g->scratch_owned && g->scratch) (void)hipFree(g->scratch);
      g->scratch_owned = false;
      detach_scratch(g);
      for (auto b : kApplyBufs) (g->*b).release();
    }
  }
  if (rc != DFPR_OK) {
    (void)hipFree(R);
    return rc;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  Resident r;
  r.g = g;
  r.R = R;
  r.scratch = sbytes;
  sv->graphs.push_back(r);
  *gid = (int32_t)sv->graphs.size() - 1;
  return DFPR_OK;
}

int server_submit(dfpr_server* sv, int32_t gid, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                  int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, double* r_out, int64_t* ticket) {
  std::unique_ptr<Request> q(new Request());
  q->gid = gid;
  q->ds.assign(del_src, del_src + n_del);
  q->dd.assign(del_dst, del_dst + n_del);
  q->is.assign(ins_src, ins_src + n_ins);
  q->id.assign(ins_dst, ins_dst + n_ins);
  q->r_out = r_out;
  q->apply_bytes = apply_buffer_bytes(n_del + n_ins, true);
  q->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (gid < 0 || gid >= (int32_t)sv->graphs.size()) {
    set_error("unknown graph id %d", gid);
    return DFPR_EINVAL;
  }
  q->ticket = sv->next_ticket++;
  *ticket = q->ticket;
  sv->queue.push_back(q.get());
  sv->requests[q->ticket] = std::move(q);
  sv->counters.submitted++;
  sv->cv_work.notify_one();
  return DFPR_OK;
}

int server_wait(dfpr_server* sv, int64_t ticket, dfpr_stats* st, dfpr_batch_info* info, double* latency_ms,
                double* queue_ms) {
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->requests.find(ticket);
  if (it == sv->requests.end()) {
    set_error("unknown or already collected ticket %lld", (long long)ticket);
    return DFPR_EINVAL;
  }
  Request* q = it->second.get();
  sv->cv_done.wait(lk, [&] { return q->done; });
  using ms = std::chrono::duration<double, std::milli>;
  if (st) *st = q->st;
  if (info) *info = q->info;
  if (latency_ms) *latency_ms = ms(q->t_done - q->t_submit).count();
  if (queue_ms) *queue_ms = ms(q->t_start - q->t_submit).count();
  const int rc = q->rc;
  if (rc != DFPR_OK) set_error("%s", q->err.c_str());
  sv->requests.erase(it);
  return rc;
}

int server_ranks(dfpr_server* sv, int32_t gid, double* r_out, dfpr_where where) {
  std::unique_lock<std::mutex> lk(sv->mu);
  if (gid < 0 || gid >= (int32_t)sv->graphs.size()) {
    set_error("unknown graph id %d", gid);
    return DFPR_EINVAL;
  }
  Resident& r = sv->graphs[gid];
  sv->cv_done.wait(lk, [&] {  // quiesce this graph: nothing queued or running for it
    if (r.busy) return false;
    for (Request* q : sv->queue)
      if (q->gid == gid) return false;
    return true;
  });
  DFPR_HIP(hipMemcpy(r_out, r.R, (size_t)r.g->n * sizeof(double),
                     where == DFPR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice));
  return DFPR_OK;
}

int server_stats(dfpr_server* sv, dfpr_server_stats* out) {
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->counters;
  out->queued = (int64_t)sv->queue.size();
  out->in_flight = sv->in_flight;
  out->graphs = (int32_t)sv->graphs.size();
  out->lanes = sv->active_lanes;
  out->heap_bytes = (int64_t)sv->heap.capacity();
  out->heap_used = (int64_t)sv->heap.used();
  out->heap_peak = (int64_t)sv->heap.peak();
  return DFPR_OK;
}

int server_set_active_lanes(dfpr_server* sv, int32_t k) {
  std::lock_guard<std::mutex> lk(sv->mu);
  if (k < 1 || k > (int32_t)sv->lanes.size()) {
    set_error("active lanes must lie in [1, %d]", (int)sv->lanes.size());
    return DFPR_EINVAL;
  }
  sv->active_lanes = k;
  sv->cv_work.notify_all();
  return DFPR_OK;
}

int32_t server_graph_n(dfpr_server* sv, int32_t gid) {
  std::lock_guard<std::mutex> lk(sv->mu);
  if (gid < 0 || gid >= (int32_t)sv->graphs.size()) return -1;
  return sv->graphs[gid].g->n;
}

}  // namespace dfpr
