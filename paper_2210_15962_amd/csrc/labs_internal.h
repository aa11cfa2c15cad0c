// labs_internal.h -- declarations shared by the host runtime and the device
// translation unit of liblabs.so.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace lsaw {

constexpr int kLMax = 383;          // D <= 192 free bits, W <= 3 key words
constexpr int kEnergyLMax = 1024;   // labs_energy: E fits int32 for any +-1 sequence
constexpr int kBlock = 256;         // threads per workgroup of the walk kernel
constexpr int kBucketBytes = 64;    // visited-table bucket (one HBM burst)

inline int free_bits(int L) { return (L + 1) / 2; }
inline int key_words_for(int L) { return (free_bits(L) + 63) / 64; }
inline int lag_words_for(int L) { return ((L - 1) / 2 + 31) / 32; }
// 16-byte entries hold keys of up to 127 bits plus an occupancy flag; longer
// keys use 32-byte entries.
inline int entry_bytes_for(int L) { return free_bits(L) <= 127 ? 16 : 32; }

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
  uint8_t *tables;          // chunk's visited tables, n_walks * table_bytes
  uint64_t table_bytes;     // bytes per walk (n_buckets * kBucketBytes)
  uint32_t n_buckets;
  int32_t lanes_per_walk;   // 1, 2, 4 or 8
};

// Device entry points (labs_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_energy(const int8_t *seqs, int32_t L, int64_t n, int32_t *E_out,
                         hipStream_t stream);
hipError_t launch_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t *out,
                         hipStream_t stream);
hipError_t launch_walks(const WalkLaunch &w, hipStream_t stream);
// Dynamic LDS bytes the walk kernel needs for length L (0 if unsupported).
size_t walk_lds_bytes(int32_t L);

}  // namespace lsaw
