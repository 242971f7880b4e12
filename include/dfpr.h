/*
 * dfpr — Dynamic Frontier PageRank on MI355X (gfx950).
 *
 * C ABI of the GPU library.  It implements the incremental PageRank update of
 * Sahu, "DF* PageRank: Improved Incrementally Expanding Approaches for Updating
 * PageRank on Dynamic Graphs" (arXiv 2401.15870): apply a batch of edge
 * deletions and insertions to a graph held in device memory, then update the
 * ranks from the previous ranks with Static, Naive-dynamic (ND), Dynamic
 * Frontier (DF) or Dynamic Frontier with Pruning (DF-P).
 *
 * Conventions shared by every call:
 *  - Every function returns an int status: DFPR_OK (0) or a negative error
 *    code.  Nothing throws across the ABI.  dfpr_last_error() returns a
 *    thread-local message describing the last failing call on this thread.
 *  - Vertex ids are int32 in [0, n).  Ranks are IEEE binary64 (FP64).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it.  dfpr_update_ranks returns only once its
 *    outputs are final; create, apply and export return once their work is
 *    complete on the stream.
 *  - Pointers marked DFPR_HOST / DFPR_DEVICE by a `where` argument point to
 *    host memory or to device memory of the current HIP device.  Input
 *    pointers are borrowed for the duration of the call only; the library
 *    copies what it keeps.
 *  - Validation happens before mutation: on DFPR_EINVAL or DFPR_ERANGE the
 *    graph is unchanged.  A HIP runtime failure returns DFPR_EHIP and poisons
 *    the handle; later calls on it return DFPR_ESTATE.
 *  - One writer per handle: calls on the same handle are serialised by an
 *    internal mutex.  Different handles may be used from different threads.
 */
#ifndef DFPR_H
#define DFPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DFPR_OK = 0,
  DFPR_EINVAL = -1, /* bad argument: null pointer with count > 0, n <= 0, bad parameter */
  DFPR_ERANGE = -2, /* a vertex id outside [0, n) */
  DFPR_ENOMEM = -3, /* device or host allocation failed; the handle stays usable */
  DFPR_EHIP = -4,   /* HIP runtime failure; the handle is poisoned */
  DFPR_ESTATE = -5  /* the handle was poisoned by an earlier failure */
};

typedef enum { DFPR_STATIC = 0, DFPR_ND = 1, DFPR_DF = 2, DFPR_DFP = 3 } dfpr_mode;
typedef enum { DFPR_HOST = 0, DFPR_DEVICE = 1 } dfpr_where;

/* Parameters of the rank update (Section 5.1.2 and Sections 4.2-4.3).
 * alpha: damping factor in (0,1).  tol: iteration tolerance on the L-inf norm
 * of the rank change (> 0).  frontier_tol (tau_f): a processed vertex marks its
 * out-neighbours when its relative change exceeds it.  prune_tol (tau_p): DF-P
 * unmarks a processed vertex whose relative change is at most this.
 * dense_switch (>= 0, may be +infinity): weight w of the choice between the
 * two forms of a DF/DF-P iteration, which give identical results and differ
 * in how an iteration's expansion reaches the next one.  The frontier form
 * pushes a mark along every out-edge of the expanding vertices; the dense form
 * processes every vertex and lets each vertex it does not keep check its
 * in-neighbours' expand flags.  An iteration runs dense when
 * |E| - (in-edges of the affected vertices) + |V| < w * (out-edges of the
 * last iteration's expanding vertices).  0 = never dense, infinity = always,
 * default 1 (a pushed mark priced like a checked flag).
 * max_iters >= 1.  flags: DFPR_FLAG_* bits.  criterion: DFPR_CRIT_*. */
typedef struct {
  double alpha, tol, frontier_tol, prune_tol, dense_switch;
  int32_t max_iters;
  int32_t flags;
  int32_t criterion; /* DFPR_CRIT_*: the change compared with frontier_tol and prune_tol */
  int32_t reserved;  /* 0 */
} dfpr_params;

/* Frontier measures of Section 4.2.  RELATIVE (the method's choice and the
 * default): |r - R[v]| / max(r, R[v]).  ABSOLUTE: |r - R[v]|.  CONTRIB: the
 * change of the contribution factor, |r - R[v]| / |out(v)|.  DF-P prunes with
 * the same measure. */
enum { DFPR_CRIT_RELATIVE = 0, DFPR_CRIT_ABSOLUTE = 1, DFPR_CRIT_CONTRIB = 2 };

/* flags: record per-phase and per-kernel timings with HIP events into dfpr_stats. */
#define DFPR_FLAG_TIMING 1
/* flags: DF and DF-P update ranks and contributions in place as vertices are
 * processed, so vertices processed later in an iteration already read the new
 * values: the asynchronous single-vector execution of Section 4.4.  Fewer
 * iterations; the result depends on the order the device happens to run in,
 * so it is not reproducible bit for bit and matches the synchronous result
 * only within the convergence tolerance.  Static and ND ignore the flag. */
#define DFPR_FLAG_ASYNC 2

/* Effective-batch counts of one dfpr_apply_batch call (Section 3.2).  The ms_*
 * fields are filled when timing is on (dfpr_set_timing), else 0. */
typedef struct {
  int64_t ins_in, ins_effective;   /* insertions given; of those, new edges      */
  int64_t del_in, del_effective;   /* deletions given; of those, removed edges   */
  int64_t self_loop_dels_ignored;  /* distinct (v,v) deletions (self-loops stay) */
  int64_t m_after;                 /* |E| after the update, self-loops included  */
  double ms_total;                 /* whole call on the stream                   */
  double ms_sort;                  /* radix sorts of the batch                   */
  double ms_rebuild[2];            /* out-CSR and in-CSR rebuild kernels         */
  int32_t row_local;               /* 1: merged into the touched rows' free slots
                                      (dfpr_set_row_slack), other rows unmoved   */
  int32_t reserved;
} dfpr_batch_info;

/* Number of in-degree bins of the pull kernel (see dfpr_set_tuning). */
#define DFPR_BINS 6

/* Result statistics of one dfpr_update_ranks call. */
typedef struct {
  int32_t iterations;              /* rank iterations run (the one that met tol counts) */
  int32_t converged;               /* 1 if the L-inf change fell to tol, 0 at max_iters */
  double last_delta;               /* L-inf rank change of the last iteration           */
  int64_t ever_affected;           /* vertices processed in at least one iteration      */
  int64_t vertex_updates;          /* sum over iterations of the affected-set size      */
  int64_t edges_pulled;            /* sum over iterations of the affected in-degrees    */
  int64_t bin_vertices[DFPR_BINS]; /* vertex_updates split by in-degree bin             */
  int64_t bin_edges[DFPR_BINS];    /* edges_pulled split by in-degree bin               */
  /* Timings in milliseconds, measured with HIP events on the stream when the
   * TIMING flag is set or timing is on for the graph (dfpr_set_timing). */
  double ms_total;                 /* the whole call                                    */
  double ms_pull;                  /* summed duration of the pull kernel launches       */
  int32_t pull_launches;           /* launches summed in ms_pull                        */
  int32_t reserved;
  double ms_commit;                /* commit + expansion kernels                        */
  double ms_bin;                   /* affected-set binning (compaction) kernels         */
  double ms_mark;                  /* initial marking kernels                           */
  /* Algorithmic bytes of all pull launches (every gather counted): frontier
   * pull 30 B per processed vertex + 12 B per pulled edge; Static/ND 36 B per
   * vertex + 12 B per edge; dense DF/DF-P pull 24 B per vertex + 8 B per
   * vertex whose rank it writes (processed, or copied over from the other
   * vector) + 5 B per edge (index + expand flag) + 8 B per pulled edge. */
  double pull_bytes;
  int32_t dense_iterations;        /* iterations run in dense (all-vertex) mode         */
  int32_t reserved2;
  /* Dense iterations run by the two-phase pull (dfpr_set_two_phase), counted
   * here and not in the pull fields above: duration of the three kernels of
   * each pass, and algorithmic bytes: 22 B per edge (index word 4, value
   * written 8, destination slot 2, value read 8) + 65 B per vertex
   * (contribution, expand flag, accumulators written and read, the update's
   * offsets, degrees, rank and flags) + 8 B per vertex whose rank it writes +
   * 4 B per pair offset loaded by each phase-one work item. */
  double ms_two_phase;
  double two_phase_bytes;
  int32_t two_phase_passes;
  int32_t reserved3;
} dfpr_stats;

typedef struct dfpr_graph dfpr_graph;

/* Paper defaults: alpha 0.85, tol 1e-10, tau_f = tau_p = 1e-6, 500 iterations
 * (Section 5.1.2; Sections 4.2-4.3); dense_switch 1. */
void dfpr_params_default(dfpr_params* p);

/* Create a graph on the current HIP device from a COO edge list of m pairs.
 * The stored graph is canonical: duplicate pairs are dropped and a self-loop is
 * added to every vertex (Sections 3.1 and 5.1.3), so |E| counts them.  The
 * handle owns all its device memory (both CSRs, their rebuild buffers and the
 * rank scratch), allocated here so that later updates allocate nothing unless a
 * batch outgrows the edge capacity.  edge_capacity (0 = automatic) reserves room
 * for that many edges.  flags: DFPR_CREATE_* bits.  Errors: EINVAL (n <= 0, m < 0, null arrays with m > 0,
 * n or m beyond int32), ERANGE (an id outside [0,n)), ENOMEM, EHIP. */
int dfpr_graph_create(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      dfpr_where where, int64_t edge_capacity, int32_t flags, void* stream,
                      dfpr_graph** out);

/* create flags.  By default the library numbers vertices internally by
 * decreasing in-degree, so that the rank contributions of the high-degree
 * vertices, which most edges read, sit together in cache; ids at the ABI are
 * always the caller's.  KEEP_IDS keeps the caller's numbering inside too
 * (then the one-lane bin sums in the caller's ascending source order). */
#define DFPR_CREATE_KEEP_IDS 1

int dfpr_graph_destroy(dfpr_graph* g);

/* |V| and |E| (self-loops included). */
int dfpr_graph_size(const dfpr_graph* g, int32_t* n, int64_t* m);

/* Copy the current canonical CSR out.  in_csr = 0: out-adjacency (row u lists
 * out(u) ascending); in_csr = 1: in-adjacency (row v lists in(v) ascending).
 * offsets has n+1 entries, indices m entries (m from dfpr_graph_size). */
int dfpr_graph_export(const dfpr_graph* g, int in_csr, int32_t* offsets, int32_t* indices,
                      dfpr_where where, void* stream);

/* Apply one batch update (Section 3.2).  Deletions and insertions are read as
 * sets: repeated pairs count once, a pair both deleted and inserted is present
 * afterwards, deleting (v,v) is ignored, inserting an existing edge or deleting
 * an absent one has no effect.  Both CSRs are rebuilt (canonical form).  The
 * sources of the effective changes and the targets of effective deletions are
 * remembered until the next DF/DF-P update, which marks out(u) of every such
 * source u in the old and new graph (Algorithm 1, initial marking).
 * info may be NULL.  Errors: EINVAL, ERANGE (graph unchanged), ENOMEM, EHIP. */
int dfpr_apply_batch(dfpr_graph* g, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                     int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst,
                     dfpr_where where, void* stream, dfpr_batch_info* info);

/* Allocation-free variant of dfpr_apply_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, effect, results and
 * errors as dfpr_apply_batch, but the batch's sort and staging buffers come
 * from a fixed scratch array inside the library (40 MiB of device memory per
 * device the library runs on, held until the process ends) and the call makes
 * no device allocation.  Limits: n_del + n_ins <= DFPR_NOALLOC_MAX_PAIRS (else
 * EINVAL), and the insertions must fit the graph's edge capacity (m + n_ins
 * <= the capacity reserved at create; else ENOMEM, where dfpr_apply_batch
 * would grow it).  The call returns once its work on the stream has finished.
 * No HIP-event timings are recorded (the info's ms_* fields stay 0).  Every
 * call on a device shares that device's scratch array: calls from one process
 * are serialised by a lock, and calls that overlap on one device from
 * different processes race. */
#define DFPR_NOALLOC_MAX_PAIRS (1 << 19)
int dfpr_apply_batch_noalloc(dfpr_graph* g, int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
                             int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where,
                             void* stream, dfpr_batch_info* info);

/* Update ranks (Algorithm 1; Equations 1 and 2).  r_prev and r_out are device
 * arrays of n doubles owned by the caller; they may alias.  STATIC ignores
 * r_prev and starts from 1/n; ND processes every vertex from r_prev; DF and
 * DF-P process the frontier grown from the pending batch marks.  Iterations are
 * synchronous: all reads of iteration i see the ranks of iteration i.  p = NULL
 * uses dfpr_params_default.  Non-convergence within max_iters is not an error
 * (stats->converged = 0).  st may be NULL.  STATIC and ND discard pending marks;
 * DF and DF-P consume them.  Errors: EINVAL (bad mode or parameters, null
 * arrays), ENOMEM, EHIP. */
int dfpr_update_ranks(dfpr_graph* g, dfpr_mode mode, const dfpr_params* p, const double* r_prev,
                      double* r_out, void* stream, dfpr_stats* st);

/* In-degree thresholds of the pull kernel.  An affected vertex v with in-degree
 * d goes to bin 0 if d <= bounds[0] (one lane per vertex, sum in ascending
 * source order), bin 1 if d <= bounds[1] (4 lanes), bin 2 if d <= bounds[2]
 * (16 lanes), bin 3 if d <= bounds[3] (one wavefront), bin 4 if d <= bounds[4]
 * (one workgroup), else bin 5 (the row split in chunks over workgroups).  The
 * bins only change performance and the summation order.  EINVAL unless
 * 1 <= bounds[0] <= ... <= bounds[4]. */
int dfpr_set_tuning(dfpr_graph* g, const int32_t bounds[5]);
int dfpr_get_tuning(const dfpr_graph* g, int32_t bounds[5]);

/* Autotuner: choose the in-degree thresholds of the pull kernel for this
 * graph by timing a few Static iterations (HIP events) for each candidate, one
 * threshold at a time (coordinate descent from the current setting; a change
 * must win by 3 %).  On a plain graph each candidate's time also includes a
 * pull over the rows of more than 128 in-edges alone, the part of the graph
 * a hub-heavy DF/DF-P frontier keeps pulling, where long rows cannot hide
 * behind other work.  The best setting is installed and written to
 * bounds_out (nullable); ms_out (nullable) receives its average Static pull
 * time.  Uses temporary device memory for one rank vector (and n bytes of
 * flags); pending batch marks are left untouched. */
int dfpr_autotune(dfpr_graph* g, void* stream, int32_t bounds_out[5], double* ms_out);

/* Graphs of at most max_edges edges (self-loops included) run a whole rank
 * update in one cooperative launch: every iteration's pull over all vertices
 * (DF/DF-P in the dense form), a grid-wide barrier, and the stopping test on
 * the device, instead of several launches and a readback per iteration.  The
 * results are the same bits either way (same kernels, same work split); only
 * the latency changes.  Default 4194304; 0 disables.  On a batch handle the
 * limit applies to the arena (default 67108864): each member converges and
 * drops out on its own inside the launch (a second grid barrier per iteration
 * folds the members' changes).  Errors: EINVAL (max_edges < 0). */
int dfpr_set_fused_limit(dfpr_graph* g, int64_t max_edges);

/* Free slots after every CSR row, so that small batches (Section 3.2) change
 * only the rows they touch.  Lays both CSRs out again with `slack` free slots
 * after the neighbours of every row (0, the default: rows packed).  Afterwards
 * a batch of at most one effective pair per 256 slots whose touched rows all
 * have room for their net insertions is merged into those rows in place:
 * offsets and all other rows stay where they are, and the apply costs the
 * touched rows plus the batch instead of a copy of both CSRs.  If some
 * touched row has no room, the apply lays every row out again with `slack`
 * fresh free slots; larger batches take the usual rebuild, which keeps each
 * row's free slots.  The rank kernels read only the neighbours.  Exports,
 * sizes and results are the same as without slack.  Each index array then
 * holds m + n * slack slots (the edge capacity grows if needed).  A served
 * graph keeps the layout it had when added.  Errors: EINVAL (slack outside
 * [0, 65536], or more slots than int32 offsets reach), ENOMEM. */
int dfpr_set_row_slack(dfpr_graph* g, int32_t slack, void* stream);

/* Dense-form iterations of DF and DF-P (Algorithm 1; Equations 1 and 2) in
 * two phases instead of one gathering pull (on = 1; 0, the default, turns it
 * off and frees its memory).  Phase one writes every edge's contribution
 * R[u]/|out(u)| into an array ordered by destination range, reading the
 * contributions of one source range at a time from LDS; phase two streams
 * each destination range once and adds into accumulators in LDS.  The sums
 * are exact: each contribution is taken as an integer multiple of 2^-96
 * (exactly, for contributions of at least 2^-44) and the 128-bit integers
 * are added, so the order of additions does not matter and each sum is
 * rounded to FP64 once.  Results are reproducible bit for bit but differ from
 * the gather pull's FP64 sums by rounding (the affected sets follow from
 * them).  The layout (14 bytes per edge: 6 of layout, 8 of values) is built
 * from the in-CSR before the first dense iteration after every change of the
 * graph.  On R-MAT graphs of 2^24 vertices a pass takes longer than the gather
 * pull and the rebuild adds to every batch, so the gather pull stays the
 * default.  Frontier-form iterations, the single-launch loop (dfpr_set_fused_limit)
 * and the asynchronous mode keep the gather pull.  Contributions must lie in
 * [0, 2^31) and in-neighbour sums below 2^32 (any rank vector with entries
 * in [0, 1] qualifies): an update with a contribution outside [0, 2^31) fails
 * with EINVAL.
 * Errors: EINVAL (batch handle, or more than 2^25 vertices). */
int dfpr_set_two_phase(dfpr_graph* g, int on);

/* Turn HIP-event timing of every apply and update on this graph on (1) or
 * off (0).  Events are recorded between kernels and read after the call's
 * final synchronisation, so timing adds no host round trips. */
int dfpr_set_timing(dfpr_graph* g, int on);

/* ---- Batched form: many independent graphs updated together.
 *
 * Graphs that each need the same update (apply a batch, then Static / ND / DF /
 * DF-P) are held as one batch handle: the disjoint union of the member graphs
 * in one device arena, member k owning the vertex range [base_k, base_k + n_k).
 * Every step of the update runs once over the whole arena, so small graphs
 * share launches instead of each paying its own.  Each member follows
 * Algorithm 1 on its own: its constant term is (1 - alpha)/n_k (Equation 1 with
 * |V| = n_k), its Static start is 1/n_k, and its L-inf change, iteration count
 * and convergence are its own; a member that has converged drops out of the
 * later iterations of the call, so its result is the one its plain-handle
 * update would give.  With the default thresholds and the same create flags the
 * results are bit-identical to per-graph plain handles.  Rank vectors of a
 * batch handle have one entry per arena vertex; member k's ranks sit at
 * [base_k, base_k + n_k) in its own vertex order.
 *
 * On a batch handle, dfpr_apply_batch is refused (EINVAL: its ids could join
 * members); dfpr_update_ranks works and reports totals only; dfpr_graph_size,
 * dfpr_graph_export and the tuning calls see the arena.
 *
 * Why an arena built at create, rather than calls over a list of existing
 * plain handles: one launch can cover many members only when their CSRs,
 * ranks and flags are one contiguous address range with one vertex numbering
 * (the bins, worklists and chunk tables of the pull span all members), and
 * gathering separately allocated graphs into such a range on every call would
 * copy every graph every step.  The member set is therefore fixed for the
 * handle's life: to add or drop members, create a new batch handle (a plain
 * handle's graph can be exported and passed in). */

/* Create a batch handle from `count` >= 1 member edge lists.  Member k has
 * n[k] >= 1 vertices and m[k] >= 0 pairs src[k][i] -> dst[k][i] with ids in
 * [0, n[k]) (all arrays in `where` memory; the pointer arrays themselves on
 * the host).  Each member is made canonical like dfpr_graph_create.  flags as
 * for dfpr_graph_create.  Errors: EINVAL (count < 1, n[k] < 1, m[k] < 0, null
 * arrays with m[k] > 0, arena beyond int32), ERANGE (an id outside its member),
 * ENOMEM, EHIP. */
int dfpr_batch_create(int32_t count, const int32_t* n, const int64_t* m, const int32_t* const* src,
                      const int32_t* const* dst, dfpr_where where, int32_t flags, void* stream,
                      dfpr_graph** out);

/* Number of members (1 for a plain handle). */
int dfpr_batch_count(const dfpr_graph* g, int32_t* count);

/* Vertex range of member k in the arena: base and n. */
int dfpr_batch_member(const dfpr_graph* g, int32_t k, int32_t* base, int32_t* n);

/* Apply one batch update to every member (Section 3.2, per member as in
 * dfpr_apply_batch).  Per member k: n_del[k] deletions del_src[k][i] ->
 * del_dst[k][i] and n_ins[k] insertions, ids member-local.  info (nullable)
 * receives `count` entries; their ms_* fields time the whole call.  Errors:
 * EINVAL, ERANGE (no member changed), ENOMEM, EHIP. */
int dfpr_apply_batch_many(dfpr_graph* g, const int64_t* n_del, const int32_t* const* del_src,
                          const int32_t* const* del_dst, const int64_t* n_ins, const int32_t* const* ins_src,
                          const int32_t* const* ins_dst, dfpr_where where, void* stream, dfpr_batch_info* info);

/* Update the ranks of every member (Algorithm 1; Equations 1 and 2 per
 * member).  r_prev / r_out: device arrays over the arena (see above), may
 * alias.  total (nullable): iterations = the most any member ran, converged =
 * all members converged, last_delta = the largest member last change,
 * ever_affected and the work counters summed, timings of the whole call.
 * per_graph (nullable, `count` entries): iterations, converged, last_delta and
 * ever_affected of each member; its other fields are 0.  Errors as for
 * dfpr_update_ranks. */
int dfpr_update_ranks_many(dfpr_graph* g, dfpr_mode mode, const dfpr_params* p, const double* r_prev,
                           double* r_out, void* stream, dfpr_stats* total, dfpr_stats* per_graph);

/* ---- Serving form: a request loop over graphs resident in HBM.
 *
 * The server owns graphs and their current ranks in device memory.  A request
 * (graph id, batch) applies the batch to that graph (Section 3.2) and updates
 * its resident ranks with the server's mode, DF-P by default (Algorithm 1 from
 * the ranks left by the previous request).  Requests for one graph run one at
 * a time in submission order (a single writer per graph, Section 3.2);
 * requests for different graphs run concurrently on `lanes` worker lanes, each
 * with its own HIP stream, so their kernels overlap on the device.  A request
 * is admitted when a lane is free, its graph is idle and its blocks (the
 * vertex arrays of one update, its batch sort buffers and the targets into
 * which both CSRs are rebuilt) can be taken from the server's device heap of
 * `heap_bytes`, reserved once at create.  The heap also holds every graph's
 * current CSRs: a request's rebuild targets become the graph's CSRs and the
 * old ones go back to the heap, so the heap bounds all graph memory but the
 * rank vectors.  Requests that do not fit wait (later ones do not overtake
 * them), so a small heap serialises work instead of failing it.  A request
 * whose blocks exceed what the heap can ever free fails with ENOMEM.
 * Single-launch updates of different lanes share the device's budget of
 * resident workgroups.  Results are those of the plain entry points: a
 * graph's ranks do not depend on what else is in flight.
 *
 * The mode and parameters are fixed at create and every graph's ranks stay
 * resident in the server (each request continues from the result of the
 * previous one on its graph, like the consecutive batch updates of Section
 * 5.1.4); a request names the host array that receives a copy of its result,
 * if any, instead of passing rank vectors in and out as dfpr_update_ranks
 * does. */
typedef struct dfpr_server dfpr_server;

typedef struct {
  int64_t submitted, completed, failed; /* requests so far                          */
  int64_t queued;                       /* waiting for admission                    */
  int64_t peak_in_flight;               /* most requests running at once            */
  int32_t in_flight, graphs, lanes, reserved;  /* lanes: active lanes */
  int64_t heap_bytes, heap_used, heap_peak;
} dfpr_server_stats;

/* Create a server on the current device: heap_bytes > 0 of scratch heap, lanes
 * in [1, 64], mode STATIC/ND/DF/DFP, p as for dfpr_update_ranks (NULL =
 * defaults).  Errors: EINVAL, ENOMEM, EHIP. */
int dfpr_server_create(size_t heap_bytes, int32_t lanes, dfpr_mode mode, const dfpr_params* p,
                       dfpr_server** out);

/* Drain every queued and running request, then free the server, its graphs and
 * their resident ranks. */
int dfpr_server_destroy(dfpr_server* sv);

/* Move a plain graph handle into the server (on success the caller must not
 * use or destroy g any more) and give it resident ranks: a copy
 * of r0 (device, n doubles) or, with r0 = NULL, a Static solve.  Its CSRs
 * move into the heap; its rebuild targets and scratch are released: from now
 * on each request borrows them from the heap.  On error the handle still
 * belongs to the caller.  Errors: EINVAL (batch handle), ENOMEM (the heap
 * cannot hold the graph's CSRs), EHIP. */
int dfpr_server_add_graph(dfpr_server* sv, dfpr_graph* g, const double* r0, int32_t* gid);

/* Queue a request: one batch (host arrays, copied before return; ids in
 * [0, n) of graph gid, read as sets as in dfpr_apply_batch).  r_out (nullable)
 * is a host array of n doubles that receives the graph's ranks after this
 * request; it must stay valid until dfpr_server_wait returns for the ticket.
 * Errors: EINVAL (unknown graph, negative counts, null arrays). */
int dfpr_server_submit(dfpr_server* sv, int32_t gid, int64_t n_del, const int32_t* del_src,
                       const int32_t* del_dst, int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst,
                       double* r_out, int64_t* ticket);

/* Wait for a request and collect it (each ticket once).  st, info, latency_ms
 * (submit to result ready) and queue_ms (submit to admission) are nullable.
 * Returns the request's own status: ERANGE (an id outside [0, n); the graph and
 * its ranks are unchanged), ENOMEM (scratch larger than the heap), ESTATE/EHIP. */
int dfpr_server_wait(dfpr_server* sv, int64_t ticket, dfpr_stats* st, dfpr_batch_info* info,
                     double* latency_ms, double* queue_ms);

/* Copy graph gid's resident ranks (n doubles, caller order) to r_out once no
 * request for it is queued or running. */
int dfpr_server_ranks(dfpr_server* sv, int32_t gid, double* r_out, dfpr_where where);

/* Vertex count of graph gid. */
int dfpr_server_graph_size(dfpr_server* sv, int32_t gid, int32_t* n);

/* Counters, heap use and the number of active lanes. */
int dfpr_server_get_stats(dfpr_server* sv, dfpr_server_stats* out);

/* Limit how many lanes take new requests (1 <= k <= lanes at create); k = 1
 * runs requests one at a time in submission order.  Running requests finish
 * on their lanes.  Errors: EINVAL. */
int dfpr_server_set_active_lanes(dfpr_server* sv, int32_t k);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* dfpr_last_error(void);

/* Library version string. */
const char* dfpr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DFPR_H */
