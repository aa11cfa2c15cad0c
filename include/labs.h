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
 * 1 <= L <= 8192 (skew-symmetric or not).
 *   seqs  device int8 [n][L], each element +1 or -1 (other values give an
 *         unspecified result; the Python binding validates them).
 *   E_out device int32 [n].
 * Errors: LABS_EINVAL if L < 1, L > 8192, n < 0 or a pointer is NULL while
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

#ifdef __cplusplus
}
#endif

#endif /* LABS_H */
