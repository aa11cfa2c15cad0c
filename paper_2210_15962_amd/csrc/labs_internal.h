// labs_internal.h -- declarations shared by the host runtime and the device
// translation unit of liblabs.so.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace lsaw {

constexpr int kLMax = 383;          // D <= 192 free bits, W <= 3 key words
constexpr int kEnergyLMax = 1024;   // labs_energy: E fits int32 for any +-1 sequence
constexpr int kBlock = 256;         // threads per workgroup of the walk kernel
constexpr int kBucketBytes = 128;   // visited-table bucket (one 128-byte line)

inline int free_bits(int L) { return (L + 1) / 2; }
inline int key_words_for(int L) { return (free_bits(L) + 63) / 64; }
inline int lag_words_for(int L) { return ((L - 1) / 2 + 31) / 32; }
// Visited-table entry formats by key length: 12-byte entries (10 per bucket)
// hold keys of up to 95 bits plus an occupancy flag, 16-byte entries (8 per
// bucket) up to 127 bits, 32-byte entries (4 per bucket) up to 255 bits.
enum : int { kE12 = 0, kE16 = 1, kE32 = 2 };
__host__ __device__ constexpr int entry_format(int key_bits) {
  return key_bits <= 95 ? kE12 : key_bits <= 127 ? kE16 : kE32;
}
inline int entry_bytes_of(int fmt) { return fmt == kE12 ? 12 : fmt == kE16 ? 16 : 32; }
inline int entry_bytes_for(int L) { return entry_bytes_of(entry_format(free_bits(L))); }

// Whole search space: keys are the L sequence bits, lags k = 1..L-1.
constexpr int kFullLMax = 255;      // W <= 4 key words, <= 8 lag words
inline int full_key_words_for(int L) { return (L + 63) / 64; }
inline int full_lag_words_for(int L) { return (L - 1 + 31) / 32; }
inline int full_entry_bytes_for(int L) { return entry_bytes_of(entry_format(L)); }

struct WalkLaunch {
  const uint64_t *starts;   // device [n][W] or nullptr (seeded starts)
  uint64_t seed;
  int32_t L;
  int64_t walk_begin;       // global index of the first walk of this chunk
  int64_t n_walks;          // walks in this chunk
  int64_t walk_len;
  uint64_t *best_seq;
  int32_t *best_E;
  int64_t *steps_done;
  uint64_t *digest;
  int16_t *trace_j;
  int32_t *trace_E;
  int64_t n_trace;
  uint32_t *cap_steps;      // [n][4] scans per plane cap, or nullptr
  uint8_t *tables;          // chunk's visited tables, n_walks * table_bytes
  uint64_t table_bytes;     // bytes per walk (n_buckets * kBucketBytes)
  uint32_t n_buckets;
  int32_t lanes_per_walk;   // 1, 2, 4 or 8
};

// Progress of one walk between launches (continuous batching): the pivot, the
// best so far, the digest chain, moves made, the predecessor and a stop flag.
struct WalkState {
  uint64_t P[4];            // skew-symmetric walks use up to three words
  uint64_t bestP[4];
  uint64_t h;
  int64_t steps;
  int32_t bestE;
  uint32_t prev_jm1;
  uint32_t trapped;
  uint32_t pad;
};

// Mixed-length batches: one persistent launch drains a device work queue of
// (instance, block of walks) items.
struct BatchInstanceDev {
  const uint64_t *starts;
  uint64_t seed;
  int64_t walk_len;
  uint64_t *best_seq;
  int32_t *best_E;
  int64_t *steps_done;
  uint64_t *digest;
  int16_t *trace_j;
  int32_t *trace_E;
  int64_t n_trace;
  uint64_t table_bytes;
  uint32_t n_buckets;
  int32_t L;
  uint8_t *tables;          // per-walk tables (walk w at + w*table_bytes), or
                            // nullptr: the workgroup's arena, cleared per item
  WalkState *state;         // per-walk progress, or nullptr (single launch)
  uint8_t *wstat;           // per-walk status across launches, or nullptr
                            // (every walk starts in this launch): 0 not
                            // started, 1 started (resume from state), 2 finished
  int64_t step_end;         // a walk stops when it has made this many moves
  uint32_t *cap_steps;      // [n_walks][4] scans per plane cap, or nullptr
};

struct BatchItemDev {
  int32_t inst;       // instance index
  int32_t code;       // (lag words << 4) | lanes per walk
  int32_t n_walks;    // walks of this block
  int32_t pad;
  int64_t walk_begin; // first walk of the block within its instance
};

struct BatchLaunch {
  const BatchItemDev *items;
  int64_t n_items;
  const BatchInstanceDev *inst;
  uint32_t *counter;      // work-queue head, zeroed by launch_batch_reset
  uint8_t *arena;         // visited tables: arena_bytes per resident workgroup
  uint64_t arena_bytes;
  // Optional (nullptr: unused).  preempt: a host word the kernel polls every
  // 64 moves; once it is nonzero, walks save their state and no further item
  // starts.  item_done: word i is set to 1 when item i ends with every walk
  // finished.  Both may live in pinned host memory.
  const uint32_t *preempt;
  uint32_t *item_done;
};

// Host helpers shared by labs_api.cpp and labs_serve.cpp.
int32_t set_error(int32_t code, const char *fmt, ...);
int32_t clear_error();
// Visited-table geometry for walk_len moves at a load factor, skew-symmetric
// or whole-space keys (false if the table would not fit 32-bit bucket indices).
bool table_geometry(int32_t L, int64_t walk_len, double load_factor, uint32_t *n_buckets,
                    uint64_t *table_bytes, bool full = false);
// Lanes per walk and load factor from the tuning table (or the default).
void tuned_plan(int32_t L, int32_t *lanes, double *load_factor);

// Device entry points (labs_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_energy(const int8_t *seqs, int32_t L, int64_t n, int32_t *E_out,
                         hipStream_t stream);
hipError_t launch_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t *out,
                         hipStream_t stream);
hipError_t launch_walks(const WalkLaunch &w, hipStream_t stream);
// Dynamic LDS bytes the walk kernel needs for length L (0 if unsupported).
size_t walk_lds_bytes(int32_t L);
// Whole-space walks (labs_full.hip): lanes per walk the kernel is built for,
// its LDS bytes for length L, and the launch (w.L is the sequence length).
int full_lanes_per_walk();
size_t full_walk_lds_bytes(int32_t L);
hipError_t launch_full_walks(const WalkLaunch &w, hipStream_t stream);
// Whole-space batches: kernel group of lag-word class nw (4: classes 1-4,
// 7: classes 5-7, 8: class 8), resident workgroups per CU, and the launch.
int full_batch_variant(int nw);
// serve: the serving form (per-walk status, stop flag, item completion words).
hipError_t full_batch_blocks_per_cu(int variant, int *blocks, bool serve = false);
hipError_t launch_full_batch(const BatchLaunch &b, int variant, int grid, hipStream_t stream,
                             bool serve = false);
// Batch kernel of lag-word class nw (2..6; class 1 runs on the class-2 kernel).
int batch_variant(int nw);
size_t batch_lds_bytes(int variant);
hipError_t batch_blocks_per_cu(int variant, int *blocks, bool serve = false);
hipError_t launch_batch_reset(uint32_t *counter, hipStream_t stream);
// serve: the serving form (per-walk status, stop flag, item completion words).
hipError_t launch_batch(const BatchLaunch &b, int variant, int grid, hipStream_t stream,
                        bool serve = false);

}  // namespace lsaw
