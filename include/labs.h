/*
 * labs.h -- C ABI of liblabs.so, an MI355X (gfx950) engine for parallel
 * self-avoiding walks (SAWs) over skew-symmetric binary sequences, the search
 * of Boskovic, Herzog & Brest, "Parallel Self-Avoiding Walks for a
 * Low-Autocorrelation Binary Sequences Problem" (arXiv 2210.15962).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status codes: every call returns int32_t, LABS_OK (0) on success, a negative
 *   LABS_E* code on failure; labs_last_error() then holds a message (thread
 *   local).  Argument errors are detected synchronously before any work is
 *   queued.  Device faults surface at the caller's stream synchronisation.
 * Ownership: the caller owns every buffer.  Pointers documented as "device"
 *   must be device memory (hipMalloc or a torch CUDA tensor); "host" pointers
 *   are ordinary host memory.  No entry point allocates device memory except
 *   labs_serve_create, which allocates its pool once.
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *   Device work is enqueued asynchronously on it.
 * Sequence length: skew-symmetric calls need odd L, 3 <= L <= labs_l_max()
 *   (Eq. 2 of the paper defines the skew-symmetric space for odd L only);
 *   even or out-of-range L returns LABS_EINVAL.
 * Packed keys: a skew-symmetric sequence is stored by its D = (L+1)/2 free
 *   bits x_1..x_D (Eq. 2: the second half follows from the first) in
 *   W = ceil(D/64) uint64 words, row-major per sequence.  Free bit x_j (which
 *   is sequence element s_j) is bit (j-1)%64 of word (j-1)/64; a set bit means
 *   -1.  Bits above D must be zero.
 * Whole search space (labs_full_*): any L with 3 <= L <= labs_full_l_max();
 *   the whole sequence is packed the same way, bit i-1 = s_i, in
 *   ceil(L/64) words, bits at L and above zero.
 */
#ifndef LABS_H
#define LABS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LABS_OK         0
#define LABS_PENDING    1
#define LABS_EINVAL    (-1)
#define LABS_ENOMEM    (-2)
#define LABS_EDEVICE   (-3)
#define LABS_EBUSY     (-4)
#define LABS_ENOTFOUND (-5)

/* Message describing the last failing call on this thread ("" if none). */
const char *labs_last_error(void);

/* Largest odd L accepted by the skew-symmetric calls (W <= 3 words). */
int32_t labs_l_max(void);

/* Number of uint64 words per packed key for length L (0 if L is invalid). */
int32_t labs_key_words(int32_t L);

/*
 * labs_energy -- Eq. 1: E(S) = sum_{k=1}^{L-1} C_k^2 with
 * C_k = sum_{i=1}^{L-k} s_i s_{i+k}, for n full sequences of any length
 * 1 <= L <= 1024 (skew-symmetric or not; every such E fits int32).
 *   seqs  device int8 [n][L], each element +1 or -1 (other values give an
 *         unspecified result; the Python binding validates them).
 *   E_out device int32 [n].
 * Errors: LABS_EINVAL if L < 1, L > 1024, n < 0 or a pointer is NULL while
 * n > 0.
 */
int32_t labs_energy(const int8_t *seqs, int32_t L, int64_t n, int32_t *E_out,
                    void *stream);

/*
 * Host helpers for the packed key layout.
 *   labs_pack_skew:   x host int8 [n][D] (+-1 free bits) -> out host uint64 [n][W].
 *   labs_unpack_skew: keys host uint64 [n][W] -> x host int8 [n][D].
 *   labs_expand_skew: x host int8 [n][D] -> s host int8 [n][L], the full
 *                     sequence by Eq. 2 (s_{D+i} = (-1)^i s_{D-i}).
 * Errors: LABS_EINVAL for invalid L, n < 0, NULL pointers, or (pack) an
 * element that is not +-1, or (unpack) a key with bits set above D.
 */
int32_t labs_pack_skew(const int8_t *x, int32_t L, int64_t n, uint64_t *out);
int32_t labs_unpack_skew(const uint64_t *keys, int32_t L, int64_t n, int8_t *x);
int32_t labs_expand_skew(const int8_t *x, int32_t L, int64_t n, int8_t *s);

/*
 * labs_starts -- the seeded uniform first pivots used when labs_walks gets
 * starts == NULL (Eq. 3 draws P_1 uniformly at random).  Word t of walk w is
 * mix64(seed + 0x9E3779B97F4A7C15 * (w*W + t + 1)) masked to the valid bits,
 * where mix64 is the SplitMix64 finaliser (Steele, Lea & Flood, 2014).
 *   out device uint64 [n_walks][W].
 */
int32_t labs_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t *out,
                    void *stream);

/* Per-walk outputs of labs_walks (all device pointers). */
typedef struct labs_walk_out {
  uint64_t *best_seq;   /* [n_walks][W]: first pivot reaching the walk's minimum */
  int32_t *best_E;      /* [n_walks]: that minimum energy (Alg. 2, strict "<") */
  int64_t *steps_done;  /* [n_walks]: moves made (< walk_len if trapped) */
  uint64_t *digest;     /* [n_walks] or NULL: mix64 chain over (j, E) per move */
  int16_t *trace_j;     /* [n_trace][walk_len] or NULL: flipped free bit j (1-based) */
  int32_t *trace_E;     /* [n_trace][walk_len] or NULL: energy after each move */
  int64_t n_trace;      /* traces are written for walks 0..n_trace-1 */
  uint32_t *cap_steps;  /* [n_walks][4] or NULL: neighbourhood scans of the walk
                           evaluated on 4, 5 or 6 C planes, or on the stored
                           per-word plane counts (one scan per move, plus the
                           last scan of a trapped walk).  The low planes suffice
                           whenever every c_t = (C_t - 1)/2 of the walks sharing
                           a wavefront fits in that many bits, so the counts
                           depend on the launch plan: a performance record that
                           lets a caller price the evaluation work actually
                           needed, not a result. */
} labs_walk_out;

/*
 * Launch plan knobs.  Results never depend on them (the visited set is exact);
 * only speed and workspace size do.
 *   lanes_per_walk : 0 = automatic (tuned table), or 1, 2, 4 or 8 lanes of a
 *                    wavefront cooperating on one walk.
 *   load_factor    : 0 = default (0.5), else maximum occupancy of a walk's
 *                    visited table, in (0, 0.9].
 *   max_concurrent : 0 = as many walks at once as the workspace holds, else an
 *                    upper bound on walks resident at once.
 */
typedef struct labs_plan {
  int32_t lanes_per_walk;
  double load_factor;
  int64_t max_concurrent;
} labs_plan;

/*
 * labs_walks_workspace_bytes -- workspace that lets labs_walks keep all
 * n_walks visited tables resident at once (plan may be NULL for defaults).
 * Smaller workspaces are accepted: walks then run in consecutive chunks.
 * labs_walks_min_workspace_bytes gives the smallest usable size.
 */
int32_t labs_walks_workspace_bytes(int32_t L, int64_t n_walks, int64_t walk_len,
                                   const labs_plan *plan, uint64_t *bytes);
int32_t labs_walks_min_workspace_bytes(int32_t L, int64_t walk_len,
                                       const labs_plan *plan, uint64_t *bytes);

/*
 * labs_walks -- n_walks independent self-avoiding walks (Eq. 3, Eq. 4,
 * Alg. 2) over the skew-symmetric space of length L.
 *   starts    device uint64 [n_walks][W] first pivots, or NULL to draw them
 *             from `seed` exactly as labs_starts does (seed is ignored when
 *             starts != NULL).
 *   walk_len  number of moves per walk (Alg. 2 moves from P_1 to P_{n+1}).
 *   At every move the walk scores all D one-bit neighbours of the pivot and
 *   moves to the lowest-energy neighbour not yet visited by this walk, ties
 *   broken to the lowest j; a walk whose D neighbours are all visited stops
 *   early.  walk_len == 0 returns each start and its energy.
 *   out       per-walk results (see labs_walk_out).
 *   workspace device scratch of ws_bytes bytes (visited tables); its contents
 *             on entry are ignored and on exit are unspecified.
 * Errors: LABS_EINVAL (bad L, n_walks < 0, walk_len < 0, NULL required
 * pointer, bad plan, workspace below the minimum), LABS_EDEVICE (launch
 * failure).
 */
int32_t labs_walks(const uint64_t *starts, int32_t L, int64_t n_walks,
                   int64_t walk_len, uint64_t seed, const labs_walk_out *out,
                   void *workspace, uint64_t ws_bytes, const labs_plan *plan,
                   void *stream);

/*
 * labs_walks_noalloc -- labs_walks for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Arguments, results, streams and errors are those of
 * labs_walks without the workspace: the visited tables live in a fixed device
 * array of LABS_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every
 * GPU it runs on until the process ends (its address is looked up on the
 * first call on each device).  The walks run in chunks of as many visited
 * tables as the array holds; a walk whose table alone is larger (see
 * labs_walks_min_workspace_bytes) returns LABS_EINVAL.  The call allocates
 * nothing.  Every call on one GPU uses the same array, and each walk clears
 * its table before use: calls that overlap in time on one GPU (other streams
 * or threads of the process) race and give undefined results, so serialise
 * them, e.g. on one stream.
 */
#define LABS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t labs_walks_noalloc(const uint64_t *starts, int32_t L, int64_t n_walks,
                           int64_t walk_len, uint64_t seed, const labs_walk_out *out,
                           const labs_plan *plan, void *stream);

/*
 * Whole search space (the sokol_full solver that Sec. 5 names as future
 * work): the walks of labs_walks over all 2^L binary sequences of any length
 * L, 3 <= L <= labs_full_l_max() (255), even or odd.  The pivot is the whole
 * sequence, packed in W = ceil(L/64) words (bit i-1 = s_i, 1 means -1, bits
 * at L and above zero); a neighbour negates one sequence position, so every
 * move scores all L neighbours by Eq. 1 (computed incrementally, exactly) and
 * moves to the lowest-energy one not yet visited, ties broken to the lowest
 * position i; a walk whose L neighbours are all visited stops early.  Best
 * tracking, digest (over (i, E) per move) and traces are as in labs_walks,
 * with trace_j holding the position i (1-based).  Seeded starts: word t of
 * walk w is mix64(seed + 0x9E3779B97F4A7C15 * (w*W + t + 1)) masked to L bits.
 *   labs_full_key_words: W for a valid L, else 0.
 *   labs_full_walks_workspace_bytes: workspace for all n_walks visited tables
 *     at once (smaller workspaces run the walks in chunks, down to one table).
 *   labs_full_walks: arguments, ownership and layout as labs_walks (device
 *     pointers, asynchronous on stream, workspace contents unspecified on
 *     exit); plan->lanes_per_walk must be 0 or 4.
 * Errors: LABS_EINVAL (L outside [3, 255], n_walks < 0, walk_len < 0 or above
 * 2^31, NULL required pointer, bad plan, workspace below one table),
 * LABS_EDEVICE (launch failure).
 */
int32_t labs_full_l_max(void);
int32_t labs_full_key_words(int32_t L);
int32_t labs_full_walks_workspace_bytes(int32_t L, int64_t n_walks, int64_t walk_len,
                                        const labs_plan *plan, uint64_t *bytes);
int32_t labs_full_walks(const uint64_t *starts, int32_t L, int64_t n_walks,
                        int64_t walk_len, uint64_t seed, const labs_walk_out *out,
                        void *workspace, uint64_t ws_bytes, const labs_plan *plan,
                        void *stream);


/*
 * Mixed-length batches (several instances of different L in one launch).
 * An instance is one labs_walks job; all instances of a batch run in a
 * single persistent launch that drains a device work queue of
 * (instance, block of walks) items.  Results are identical to running each
 * instance alone with labs_walks.
 *   lanes_per_walk : 0 = tuned table (labs_tune_set / labs_autotune) or the
 *                    built-in default, else 2, 4 or 8.
 *   load_factor    : 0 = tuned table or 0.5, else in (0, 0.9].
 *   starts         : device [n_walks][W] or NULL (seeded from `seed`).
 *   out            : per-instance outputs as for labs_walks (device pointers).
 */
typedef struct labs_instance {
  int32_t L;
  int32_t lanes_per_walk;
  int64_t n_walks;
  int64_t walk_len;
  uint64_t seed;
  const uint64_t *starts;
  double load_factor;
  labs_walk_out out;
} labs_instance;

/*
 * labs_batch_workspace_bytes -- workspace for labs_walks_batch /
 * labs_batch_graph_create: queue heads, the work-item list and one visited-
 * table arena slice per resident workgroup of the current device (queries the
 * device; LABS_EDEVICE without one).  A batch runs as one persistent launch
 * per group of lag-word classes of equal occupancy; with this size the groups
 * run one after another.  A workspace with a slice for every resident
 * workgroup of every group at once lets the groups run concurrently (on
 * library-owned side streams forked from and joined back to `stream`);
 * smaller workspaces run with fewer resident workgroups.
 */
int32_t labs_batch_workspace_bytes(const labs_instance *inst, int32_t n_inst, uint64_t *bytes);

/*
 * labs_walks_batch -- run every instance (host array inst[0..n_inst-1]) in
 * persistent launches (one per class group, see above) on `stream`.  The
 * work-item list is copied into the workspace asynchronously, through a ring
 * of four pinned host buffers per device that the library keeps for the
 * process: the call returns without waiting on `stream`, except that it
 * waits for the upload of the fourth batch call before it on the device to
 * complete before reusing that buffer.  The first calls (and a call with a
 * longer list than any before) allocate pinned host memory.  The call is not
 * meant for stream capture: use labs_batch_graph_* for graphs.
 * Errors: LABS_EINVAL (any invalid instance, workspace below one arena),
 * LABS_EDEVICE.
 */
int32_t labs_walks_batch(const labs_instance *inst, int32_t n_inst, void *workspace,
                         uint64_t ws_bytes, void *stream);

/*
 * Whole-space batches (Sec. 5's sokol_full, see labs_full_walks): instances of
 * any L in [3, 255], each one labs_full_walks job (lanes_per_walk 0 or 4,
 * load_factor 0 = 0.5), run the way labs_walks_batch runs skew-symmetric
 * instances: persistent launches, one per group of lag-word classes (classes
 * 1-4, 5-7 and 8, i.e. L <= 129, L <= 225 and above), draining a work queue of
 * (instance, block of 64 walks) items, longest L first.  Workspace, streams
 * and the work-list upload behave as for labs_batch_workspace_bytes and
 * labs_walks_batch.  Results are identical to running each instance alone
 * with labs_full_walks.
 * Errors: LABS_EINVAL (any invalid instance, workspace below one arena),
 * LABS_EDEVICE.
 */
int32_t labs_full_batch_workspace_bytes(const labs_instance *inst, int32_t n_inst, uint64_t *bytes);
int32_t labs_full_walks_batch(const labs_instance *inst, int32_t n_inst, void *workspace,
                              uint64_t ws_bytes, void *stream);

/*
 * hipGraph form of labs_walks_batch: create uploads the work items once and
 * captures the queue reset and the persistent launch into an executable
 * graph; launch replays it on `stream` (each replay recomputes the same
 * results into the same output buffers); destroy releases the graph.
 */
typedef struct labs_batch_graph labs_batch_graph;
int32_t labs_batch_graph_create(const labs_instance *inst, int32_t n_inst, void *workspace,
                                uint64_t ws_bytes, labs_batch_graph **graph);
int32_t labs_batch_graph_launch(labs_batch_graph *graph, void *stream);
int32_t labs_batch_graph_destroy(labs_batch_graph *graph);

/*
 * Launch-plan tuning per L (results never depend on it).
 *   labs_tune_set / labs_tune_get : the process-wide table used when
 *     lanes_per_walk / load_factor are 0 (get returns LABS_ENOTFOUND if L has
 *     no entry, and the built-in default in the outputs).
 *   labs_autotune : times lanes_per_walk in {2, 4, 8} and load factors
 *     {0.5, 0.67} on a short run of n_walks x walk_len seeded walks (one
 *     instance through labs_walks_batch, i.e. on the batch kernel that runs
 *     batches and served requests), stores the fastest in the table and
 *     returns it.  n_walks should fill the GPU
 *     at 2 lanes per walk (about 131,072 walks on 256 CUs), else the timing
 *     measures fill rather than cost per step.  The workspace must hold
 *     labs_walks_workspace_bytes(L, n_walks, walk_len, lanes 2, load factor
 *     0.5) plus n_walks * (8W + 12) bytes rounded up to 256 (result buffers of
 *     the timing runs).  Blocks the calling thread (synchronises `stream`).
 */
int32_t labs_tune_set(int32_t L, int32_t lanes_per_walk, double load_factor);
int32_t labs_tune_get(int32_t L, int32_t *lanes_per_walk, double *load_factor);
int32_t labs_autotune(int32_t L, int64_t n_walks, int64_t walk_len, void *workspace,
                      uint64_t ws_bytes, void *stream, int32_t *best_lanes,
                      double *best_load_factor);


/*
 * Serving: a long-lived server accepts walk requests of any L as they arrive
 * and runs them with continuous batching.  A scheduler thread admits queued
 * requests first-come first-served while its device pool has room for their
 * footprint (visited tables, per-walk progress, outputs), then relaunches the
 * batch kernel over the unfinished walks of every admitted request, oldest
 * request first.  By default (chunk_steps = 0) a launch runs until its walks
 * finish or until the scheduler stops it, which it does as soon as a queued
 * request can be admitted or a running request has finished: the kernel polls
 * a stop flag in pinned host memory every 64 moves, the walks save their
 * state, and the next launch resumes them with the newcomers.  With
 * chunk_steps > 0 every launch instead advances each request by at most
 * chunk_steps moves.  Walk state and visited tables stay in device memory
 * between launches; a finished request is delivered and its memory reused at
 * once.  Each request's results equal a standalone labs_walks run with the
 * same (L, n_walks, walk_len, seed / starts) -- or, on a whole-space server
 * (labs_serve_cfg.whole_space = 1), a standalone labs_full_walks run.
 */
typedef struct labs_server labs_server;

typedef struct labs_serve_cfg {
  uint64_t pool_bytes;     /* device pool (allocated once by create); 0 = 50% of free memory */
  int32_t max_pending;     /* host queue capacity; 0 = 4096 */
  int32_t lanes_per_walk;  /* 2, 4 or 8; 0 = per launch, 4 or 8, whichever fills the
                              resident workgroups in whole rounds better */
  int64_t chunk_steps;     /* moves per launch per request; 0 = no limit (launches
                              end when a request can be admitted or has finished) */
  double load_factor;      /* visited-table load factor; 0 = default 0.5 */
  int32_t whole_space;     /* 1: the server takes whole-space requests (L in [3, 255],
                              any parity; keys as for labs_full_walks, four lanes per
                              walk); 0: skew-symmetric requests */
} labs_serve_cfg;

typedef struct labs_serve_result {
  uint64_t *best_seq;      /* host [n_walks][W] or NULL (caller-owned) */
  int32_t *best_E;         /* host [n_walks] or NULL */
  int64_t *steps_done;     /* host [n_walks] or NULL */
  uint64_t *digest;        /* host [n_walks] or NULL */
  int64_t t_submit_ns;     /* steady-clock times of submit, first launch, completion */
  int64_t t_admit_ns;
  int64_t t_done_ns;
  int64_t total_steps;     /* sum of steps_done over the request's walks */
} labs_serve_result;

typedef struct labs_serve_counters {
  int64_t submitted, admitted, completed, pending, active, launches;
  int64_t walk_steps;      /* moves made by completed requests */
  int64_t busy_ns;         /* time the device spent in the server's launches */
  uint64_t pool_bytes, pool_used, pool_peak;
} labs_serve_counters;

/* create: allocates the pool and starts the scheduler thread on the current
 * device.  destroy: stops the thread after the launch in flight, drops
 * unfinished requests and frees the pool. */
int32_t labs_serve_create(const labs_serve_cfg *cfg, labs_server **server);
int32_t labs_serve_destroy(labs_server *server);

/*
 * submit: queue one request (non-blocking).  starts is a host array
 * [n_walks][W] that is copied, or NULL for seeded starts (W and the key
 * layout of labs_walks, or of labs_full_walks on a whole-space server).  Returns LABS_EBUSY
 * when the host queue is full, LABS_EINVAL for invalid arguments or a request
 * whose footprint exceeds the whole pool.
 */
int32_t labs_serve_submit(labs_server *server, int32_t L, int64_t n_walks, int64_t walk_len,
                          uint64_t seed, const uint64_t *starts, uint64_t *req_id);

/*
 * poll: LABS_PENDING while the request runs; LABS_OK once done, after copying
 * its results into the caller's host arrays (the request is then released);
 * LABS_ENOTFOUND for an unknown or already released id.
 * wait: like poll but blocks up to timeout_ns (LABS_PENDING on timeout).
 */
int32_t labs_serve_poll(labs_server *server, uint64_t req_id, labs_serve_result *res);
int32_t labs_serve_wait(labs_server *server, uint64_t req_id, int64_t timeout_ns,
                        labs_serve_result *res);
int32_t labs_serve_stats(labs_server *server, labs_serve_counters *stats);

/*
 * Solver driver (Alg. 1): rounds of parallel walks from fresh random first
 * pivots until a stopping condition holds, keeping the global best.  Round r
 * runs walks_per_round walks of walk_len moves whose starts are walks
 * r*walks_per_round .. (r+1)*walks_per_round-1 of the labs_starts stream of
 * `seed`, so a run is reproducible and no start repeats.  After each round
 * only the per-walk best energies are copied to the host; a sequence is
 * copied only when it improves the global best.  NFEs grow by
 * walks_per_round * walk_len * (D - 1) per round, as Alg. 1 counts them.
 *   walks_per_round : > 0.
 *   walk_len        : moves per walk; 0 = 8 D (the walk length the paper uses).
 *   time_limit_s    : stop when the elapsed time reaches it (t_lmt); 0 = none.
 *   nses_limit      : stop when NFEs reach it (Eq. 6 gives one); 0 = none.
 *   target_E        : stop as soon as the best energy is <= target_E; 0 = none.
 *   max_rounds      : 0 = unlimited (then one of the limits above must be set).
 *   plan            : as for labs_walks (NULL fields = defaults).
 *   first_round     : index of this call's first round (>= 0; 0 for a fresh
 *                     run).  Rounds are deterministic in (seed, round), so a
 *                     run stopped after r rounds resumes with first_round = r:
 *                     taking the lower best_E of the two calls (the earlier
 *                     call's on ties) and summing NFEs and walk steps gives
 *                     the results of one uninterrupted run.
 * Results: best_E, best_seq (W words, packed as labs_walks), rounds run,
 * NFEs, walk steps made, seconds elapsed, and the time and NFEs at which
 * target_E was first reached (reached_target = 1), else -1.
 * workspace: labs_solve_workspace_bytes bytes of device memory.  Blocks the
 * calling thread (synchronises `stream` every round).
 * Errors: LABS_EINVAL (bad L or configuration, no stopping condition,
 * workspace too small), LABS_EDEVICE.
 */
typedef struct labs_solve_cfg {
  int64_t walks_per_round;
  int64_t walk_len;
  uint64_t seed;
  double time_limit_s;
  double nses_limit;
  int32_t target_E;
  int32_t pad;
  int64_t max_rounds;
  labs_plan plan;
  int64_t first_round;
} labs_solve_cfg;

typedef struct labs_solve_result {
  int32_t best_E;
  int32_t reached_target;
  uint64_t best_seq[3];
  int64_t rounds;
  double nfes;
  double walk_steps;
  double seconds;
  double target_seconds;   /* -1 if the target was not reached */
  double target_nfes;      /* -1 if the target was not reached */
} labs_solve_result;

int32_t labs_solve_workspace_bytes(int32_t L, const labs_solve_cfg *cfg, uint64_t *bytes);
int32_t labs_solve(int32_t L, const labs_solve_cfg *cfg, void *workspace, uint64_t ws_bytes,
                   void *stream, labs_solve_result *res);

/*
 * Stopping model of Sec. 4 (host arithmetic).  The solution evaluations one
 * run needs to reach a known optimum are exponentially distributed with rate
 * lambda(L) = 0.006753 * 0.8617^L (the trend the paper fits over L = 71..119).
 *   labs_lambda_model(L)                    : lambda(L).
 *   labs_nses_limit(L, P, N)                : Eq. 6, NSEs per run so that N
 *                                             runs reach the optimum with
 *                                             probability P: ln(1-P)/(-lambda N).
 *   labs_optimality_probability(L, nses)    : Eq. 7, 1 - exp(-lambda * nses),
 *                                             nses summed over the runs.
 * Invalid arguments (L < 1, P outside (0, 1), N < 1, nses < 0) return NaN.
 */
double labs_lambda_model(int32_t L);
double labs_nses_limit(int32_t L, double P, int32_t N);
double labs_optimality_probability(int32_t L, double nses_total);

#ifdef __cplusplus
}
#endif

#endif /* LABS_H */
