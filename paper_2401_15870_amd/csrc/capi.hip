// extern "C" entry points of libdfpr: argument validation, the per-handle
// mutex, device selection and handle poisoning around the implementation.
#include <cmath>
#include <new>

#include "dfpr_impl.hpp"

using namespace dfpr;

namespace {

// Run `fn` with the handle's device current; poison the handle on HIP failures.
template <class Fn>
int guarded(dfpr_graph* g, Fn&& fn) {
  if (!g) {
    set_error("null graph handle");
    return DFPR_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g->mu);
  if (g->poisoned) {
    set_error("graph handle is unusable after an earlier HIP failure");
    return DFPR_ESTATE;
  }
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return DFPR_EHIP;
  }
  if (prev != g->device && hipSetDevice(g->device) != hipSuccess) {
    set_error("hipSetDevice(%d) failed", g->device);
    return DFPR_EHIP;
  }
  int rc;
  try {
    rc = fn();
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    rc = DFPR_ENOMEM;
  } catch (...) {
    set_error("unexpected exception");
    rc = DFPR_EHIP;
  }
  if (rc == DFPR_EHIP) g->poisoned = true;
  if (prev != g->device) (void)hipSetDevice(prev);
  return rc;
}

int check_params(const dfpr_params& p) {
  if (!(p.alpha > 0.0 && p.alpha < 1.0)) {
    set_error("alpha must lie in (0,1), got %g", p.alpha);
    return DFPR_EINVAL;
  }
  if (!(p.tol > 0.0) || std::isnan(p.frontier_tol) || std::isnan(p.prune_tol) || !(p.dense_switch >= 0.0)) {
    set_error("tol must be > 0, dense_switch >= 0 and tolerances must not be NaN");
    return DFPR_EINVAL;
  }
  if (p.criterion < DFPR_CRIT_RELATIVE || p.criterion > DFPR_CRIT_CONTRIB) {
    set_error("unknown frontier criterion %d", p.criterion);
    return DFPR_EINVAL;
  }
  if (p.max_iters < 1) {
    set_error("max_iters must be >= 1, got %d", p.max_iters);
    return DFPR_EINVAL;
  }
  return DFPR_OK;
}

}  // namespace

extern "C" {

void dfpr_params_default(dfpr_params* p) {
  if (!p) return;
  p->alpha = 0.85;
  p->tol = 1e-10;
  p->frontier_tol = 1e-6;
  p->prune_tol = 1e-6;
  p->dense_switch = 1.0;
  p->max_iters = 500;
  p->flags = 0;
  p->criterion = DFPR_CRIT_RELATIVE;
  p->reserved = 0;
}

const char* dfpr_last_error(void) { return last_error(); }

const char* dfpr_version(void) { return "dfpr 0.1 (gfx950)"; }

int dfpr_graph_create(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, dfpr_where where,
                      int64_t edge_capacity, int32_t flags, void* stream, dfpr_graph** out) {
  clear_error();
  if (!out) {
    set_error("out is null");
    return DFPR_EINVAL;
  }
  *out = nullptr;
  if (n <= 0 || m < 0 || (m > 0 && (!src || !dst)) || (where != DFPR_HOST && where != DFPR_DEVICE) ||
      edge_capacity < 0 || (flags & ~DFPR_CREATE_KEEP_IDS) != 0) {
    set_error("invalid arguments: n=%d m=%lld", n, (long long)m);
    return DFPR_EINVAL;
  }
  try {
    return graph_create(n, m, src, dst, where, edge_capacity, flags, (hipStream_t)stream, out);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DFPR_ENOMEM;
  }
}

int dfpr_graph_destroy(dfpr_graph* g) {
  clear_error();
  if (!g) return DFPR_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != g->device) (void)hipSetDevice(g->device);
  const int dev = g->device;
  graph_destroy(g);
  if (prev != dev) (void)hipSetDevice(prev);
  return DFPR_OK;
}

int dfpr_graph_size(const dfpr_graph* g, int32_t* n, int64_t* m) {
  clear_error();
  if (!g || !n || !m) {
    set_error("null argument");
    return DFPR_EINVAL;
  }
  *n = g->n;
  *m = g->m;
  return DFPR_OK;
}

int dfpr_graph_export(const dfpr_graph* g, int in_csr, int32_t* offsets, int32_t* indices, dfpr_where where,
                      void* stream) {
  clear_error();
  if (!offsets || (!indices && g && g->m > 0) || (where != DFPR_HOST && where != DFPR_DEVICE)) {
    set_error("null output array");
    return DFPR_EINVAL;
  }
  dfpr_graph* gm = const_cast<dfpr_graph*>(g);
  return guarded(gm, [&] { return graph_export(gm, in_csr, offsets, indices, where, (hipStream_t)stream); });
}

int dfpr_apply_batch(dfpr_graph* g, int64_t n_del, const int32_t* del_src, const int32_t* del_dst, int64_t n_ins,
                     const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where, void* stream,
                     dfpr_batch_info* info) {
  clear_error();
  if (n_del < 0 || n_ins < 0 || (n_del > 0 && (!del_src || !del_dst)) || (n_ins > 0 && (!ins_src || !ins_dst)) ||
      (where != DFPR_HOST && where != DFPR_DEVICE)) {
    set_error("invalid batch arguments");
    return DFPR_EINVAL;
  }
  return guarded(g, [&] {
    if (g->ngraphs > 1) {
      set_error("batch handle: use dfpr_apply_batch_many");
      return (int)DFPR_EINVAL;
    }
    return graph_apply(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, where, (hipStream_t)stream, info);
  });
}

int dfpr_apply_batch_noalloc(dfpr_graph* g, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                             int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where,
                             void* stream, dfpr_batch_info* info) {
  clear_error();
  if (n_del < 0 || n_ins < 0 || (n_del > 0 && (!del_src || !del_dst)) || (n_ins > 0 && (!ins_src || !ins_dst)) ||
      (where != DFPR_HOST && where != DFPR_DEVICE)) {
    set_error("invalid batch arguments");
    return DFPR_EINVAL;
  }
  if (n_del + n_ins > DFPR_NOALLOC_MAX_PAIRS) {
    set_error("allocation-free apply: %lld batch pairs exceed the limit of %d", (long long)(n_del + n_ins),
              DFPR_NOALLOC_MAX_PAIRS);
    return DFPR_EINVAL;
  }
  return guarded(g, [&] {
    if (g->ngraphs > 1) {
      set_error("batch handle: use dfpr_apply_batch_many");
      return (int)DFPR_EINVAL;
    }
    return graph_apply_noalloc(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, where, (hipStream_t)stream,
                               info);
  });
}

int dfpr_update_ranks(dfpr_graph* g, dfpr_mode mode, const dfpr_params* p, const double* r_prev, double* r_out,
                      void* stream, dfpr_stats* st) {
  clear_error();
  dfpr_params prm;
  if (p) prm = *p; else dfpr_params_default(&prm);
  if (mode < DFPR_STATIC || mode > DFPR_DFP) {
    set_error("unknown mode %d", (int)mode);
    return DFPR_EINVAL;
  }
  if (check_params(prm) != DFPR_OK) return DFPR_EINVAL;
  if (!r_out || (mode != DFPR_STATIC && !r_prev)) {
    set_error("rank arrays must not be null");
    return DFPR_EINVAL;
  }
  return guarded(g, [&] { return update_ranks(g, mode, prm, r_prev, r_out, (hipStream_t)stream, st); });
}

int dfpr_batch_create(int32_t count, const int32_t* n, const int64_t* m, const int32_t* const* src,
                      const int32_t* const* dst, dfpr_where where, int32_t flags, void* stream, dfpr_graph** out) {
  clear_error();
  if (!out) {
    set_error("out is null");
    return DFPR_EINVAL;
  }
  *out = nullptr;
  if (count < 1 || !n || !m || !src || !dst || (where != DFPR_HOST && where != DFPR_DEVICE) ||
      (flags & ~DFPR_CREATE_KEEP_IDS) != 0) {
    set_error("invalid batch arguments: count=%d", count);
    return DFPR_EINVAL;
  }
  for (int32_t k = 0; k < count; k++) {
    if (n[k] < 1 || m[k] < 0 || (m[k] > 0 && (!src[k] || !dst[k]))) {
      set_error("member %d: invalid n=%d m=%lld or null arrays", k, n[k], (long long)m[k]);
      return DFPR_EINVAL;
    }
  }
  try {
    return batch_create(count, n, m, src, dst, where, flags, (hipStream_t)stream, out);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DFPR_ENOMEM;
  }
}

int dfpr_batch_count(const dfpr_graph* g, int32_t* count) {
  clear_error();
  if (!g || !count) {
    set_error("null argument");
    return DFPR_EINVAL;
  }
  *count = g->ngraphs;
  return DFPR_OK;
}

int dfpr_batch_member(const dfpr_graph* g, int32_t k, int32_t* base, int32_t* n) {
  clear_error();
  if (!g || !base || !n || k < 0 || k >= g->ngraphs) {
    set_error("null argument or member index out of range");
    return DFPR_EINVAL;
  }
  *base = (int32_t)g->vbase[k];
  *n = (int32_t)(g->vbase[k + 1] - g->vbase[k]);
  return DFPR_OK;
}

int dfpr_apply_batch_many(dfpr_graph* g, const int64_t* n_del, const int32_t* const* del_src,
                          const int32_t* const* del_dst, const int64_t* n_ins, const int32_t* const* ins_src,
                          const int32_t* const* ins_dst, dfpr_where where, void* stream, dfpr_batch_info* info) {
  clear_error();
  if (!n_del || !n_ins || (where != DFPR_HOST && where != DFPR_DEVICE)) {
    set_error("invalid batch arguments");
    return DFPR_EINVAL;
  }
  return guarded(g, [&] {
    for (int32_t k = 0; k < g->ngraphs; k++) {
      if (n_del[k] < 0 || n_ins[k] < 0 || (n_del[k] > 0 && (!del_src || !del_dst || !del_src[k] || !del_dst[k])) ||
          (n_ins[k] > 0 && (!ins_src || !ins_dst || !ins_src[k] || !ins_dst[k]))) {
        set_error("member %d: invalid batch counts or null arrays", k);
        return (int)DFPR_EINVAL;
      }
    }
    return batch_apply(g, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, where, (hipStream_t)stream, info);
  });
}

int dfpr_update_ranks_many(dfpr_graph* g, dfpr_mode mode, const dfpr_params* p, const double* r_prev,
                           double* r_out, void* stream, dfpr_stats* total, dfpr_stats* per_graph) {
  clear_error();
  dfpr_params prm;
  if (p) prm = *p; else dfpr_params_default(&prm);
  if (mode < DFPR_STATIC || mode > DFPR_DFP) {
    set_error("unknown mode %d", (int)mode);
    return DFPR_EINVAL;
  }
  if (check_params(prm) != DFPR_OK) return DFPR_EINVAL;
  if (!r_out || (mode != DFPR_STATIC && !r_prev)) {
    set_error("rank arrays must not be null");
    return DFPR_EINVAL;
  }
  return guarded(g, [&] {
    const int rc = update_ranks(g, mode, prm, r_prev, r_out, (hipStream_t)stream, total, per_graph);
    if (rc == DFPR_OK && per_graph && g->ngraphs == 1 && total) {
      per_graph[0] = dfpr_stats{};
      per_graph[0].iterations = total->iterations;
      per_graph[0].converged = total->converged;
      per_graph[0].last_delta = total->last_delta;
      per_graph[0].ever_affected = total->ever_affected;
    }
    return rc;
  });
}

int dfpr_server_create(size_t heap_bytes, int32_t lanes, dfpr_mode mode, const dfpr_params* p, dfpr_server** out) {
  clear_error();
  if (!out) {
    set_error("out is null");
    return DFPR_EINVAL;
  }
  *out = nullptr;
  dfpr_params prm;
  if (p) prm = *p; else dfpr_params_default(&prm);
  if (heap_bytes == 0 || lanes < 1 || lanes > 64 || mode < DFPR_STATIC || mode > DFPR_DFP) {
    set_error("invalid server arguments: heap_bytes=%zu lanes=%d mode=%d", heap_bytes, lanes, (int)mode);
    return DFPR_EINVAL;
  }
  if (check_params(prm) != DFPR_OK) return DFPR_EINVAL;
  try {
    return server_create(heap_bytes, lanes, mode, prm, out);
  } catch (const std::exception&) {
    set_error("server creation failed (host resources)");
    return DFPR_ENOMEM;
  }
}

int dfpr_server_destroy(dfpr_server* sv) {
  clear_error();
  if (!sv) return DFPR_OK;
  return server_destroy(sv);
}

int dfpr_server_add_graph(dfpr_server* sv, dfpr_graph* g, const double* r0, int32_t* gid) {
  clear_error();
  if (!sv || !g || !gid) {
    set_error("null argument");
    return DFPR_EINVAL;
  }
  if (g->poisoned) {
    set_error("graph handle is unusable after an earlier HIP failure");
    return DFPR_ESTATE;
  }
  try {
    return server_add_graph(sv, g, r0, gid);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DFPR_ENOMEM;
  }
}

int dfpr_server_submit(dfpr_server* sv, int32_t gid, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                       int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, double* r_out,
                       int64_t* ticket) {
  clear_error();
  if (!sv || !ticket || n_del < 0 || n_ins < 0 || (n_del > 0 && (!del_src || !del_dst)) ||
      (n_ins > 0 && (!ins_src || !ins_dst))) {
    set_error("invalid request arguments");
    return DFPR_EINVAL;
  }
  try {
    return server_submit(sv, gid, n_del, del_src, del_dst, n_ins, ins_src, ins_dst, r_out, ticket);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DFPR_ENOMEM;
  }
}

int dfpr_server_wait(dfpr_server* sv, int64_t ticket, dfpr_stats* st, dfpr_batch_info* info, double* latency_ms,
                     double* queue_ms) {
  clear_error();
  if (!sv) {
    set_error("null server");
    return DFPR_EINVAL;
  }
  return server_wait(sv, ticket, st, info, latency_ms, queue_ms);
}

int dfpr_server_ranks(dfpr_server* sv, int32_t gid, double* r_out, dfpr_where where) {
  clear_error();
  if (!sv || !r_out || (where != DFPR_HOST && where != DFPR_DEVICE)) {
    set_error("invalid arguments");
    return DFPR_EINVAL;
  }
  return server_ranks(sv, gid, r_out, where);
}

int dfpr_server_graph_size(dfpr_server* sv, int32_t gid, int32_t* n) {
  clear_error();
  if (!sv || !n) {
    set_error("null argument");
    return DFPR_EINVAL;
  }
  const int32_t v = server_graph_n(sv, gid);
  if (v < 0) {
    set_error("unknown graph id %d", gid);
    return DFPR_EINVAL;
  }
  *n = v;
  return DFPR_OK;
}

int dfpr_server_get_stats(dfpr_server* sv, dfpr_server_stats* out) {
  clear_error();
  if (!sv || !out) {
    set_error("null argument");
    return DFPR_EINVAL;
  }
  return server_stats(sv, out);
}

int dfpr_server_set_active_lanes(dfpr_server* sv, int32_t k) {
  clear_error();
  if (!sv) {
    set_error("null server");
    return DFPR_EINVAL;
  }
  return server_set_active_lanes(sv, k);
}

int dfpr_set_tuning(dfpr_graph* g, const int32_t bounds[5]) {
  clear_error();
  if (!bounds) {
    set_error("bounds is null");
    return DFPR_EINVAL;
  }
  return guarded(g, [&] {
    bool ok = bounds[0] >= 1;
    for (int i = 1; i < 5; i++) ok = ok && bounds[i] >= bounds[i - 1];
    if (!ok) {
      set_error("need 1 <= bounds[0] <= ... <= bounds[4]");
      return (int)DFPR_EINVAL;
    }
    for (int i = 0; i < 5; i++) {
      if (g->bounds[i] != bounds[i]) g->all_bins_valid = false;
      g->bounds[i] = bounds[i];
    }
    return (int)DFPR_OK;
  });
}

int dfpr_autotune(dfpr_graph* g, void* stream, int32_t bounds_out[5], double* ms_out) {
  clear_error();
  return guarded(g, [&] { return autotune(g, (hipStream_t)stream, bounds_out, ms_out); });
}

int dfpr_set_row_slack(dfpr_graph* g, int32_t slack, void* stream) {
  clear_error();
  return guarded(g, [&] { return graph_set_row_slack(g, slack, (hipStream_t)stream); });
}

int dfpr_set_two_phase(dfpr_graph* g, int on) {
  clear_error();
  return guarded(g, [&] {
    if (!on) {
      delete g->tp;
      g->tp = nullptr;
      return (int)DFPR_OK;
    }
    const char* why = nullptr;
    if (!tp_supported(g, &why)) {
      set_error("%s", why);
      return (int)DFPR_EINVAL;
    }
    if (!g->tp) g->tp = new TwoPhase();
    g->tp->on = true;
    return (int)DFPR_OK;
  });
}

int dfpr_set_fused_limit(dfpr_graph* g, int64_t max_edges) {
  clear_error();
  if (max_edges < 0) {
    set_error("max_edges must be >= 0");
    return DFPR_EINVAL;
  }
  return guarded(g, [&] {
    g->fused_limit = max_edges;
    return (int)DFPR_OK;
  });
}

int dfpr_set_timing(dfpr_graph* g, int on) {
  clear_error();
  return guarded(g, [&] {
    g->timing = on != 0;
    return (int)DFPR_OK;
  });
}

int dfpr_get_tuning(const dfpr_graph* g, int32_t bounds[5]) {
  clear_error();
  if (!g || !bounds) {
    set_error("null argument");
    return DFPR_EINVAL;
  }
  for (int i = 0; i < 5; i++) bounds[i] = g->bounds[i];
  return DFPR_OK;
}

}  // extern "C"
