// Binned splat of the RF deposit histogram (time-of-flight deposits with the
// linear tent of the path contributions, Sec. 2.3.4): the secondary-ray kernel
// records each deposit (row and bin in one key, the two tent weights); here
// the records are grouped by RF row with a counting sort whose per-block
// histograms and cursors live in LDS (each moved record is one 16-byte store:
// the scattered stores, not the arithmetic, bound this pass), and then one
// block per row and time tile
// sums its deposits in an LDS copy of the tile (fixed-point units, integer LDS
// atomics: the order of the additions does not matter) and adds the tile to
// the histogram in HBM with plain coalesced accesses. Global atomics are
// left to deposits that did not fit the record buffer.
#include "kernels.h"
#include "fir.h"

namespace usrt {

namespace {

constexpr int kBinBlocks = 256;    // blocks of the counting and scatter passes
constexpr int kBinThreads = 1024;
constexpr int kAccTile = 8192;     // samples per accumulation block (64 KB of LDS)

struct BinScratch {
  uint32_t* hist;       // [n_rows][kBinBlocks]: counts, then row start + prefix over blocks
  uint32_t* total;      // [n_rows]
  uint32_t* row_begin;  // [n_rows + 1]
};

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline BinScratch carve(void* base, int n_rows) {
  char* p = (char*)base;
  BinScratch b;
  b.hist = (uint32_t*)p;
  p += align256((size_t)kBinBlocks * n_rows * sizeof(uint32_t));
  b.total = (uint32_t*)p;
  p += align256((size_t)n_rows * sizeof(uint32_t));
  b.row_begin = (uint32_t*)p;
  return b;
}

// Records [b0, b1) of this block: kBinBlocks / kDepShards blocks split each
// shard's recorded records evenly.
constexpr int kBlocksPerShard = kBinBlocks / kDepShards;
static_assert(kBinBlocks % kDepShards == 0, "blocks per shard");

__device__ __forceinline__ void block_range(const unsigned long long* shard_count, long shard_cap, long* b0,
                                            long* b1) {
  const int shard = blockIdx.x / kBlocksPerShard, part = blockIdx.x % kBlocksPerShard;
  const long n = min((long)shard_count[shard], shard_cap);
  const long per = (n + kBlocksPerShard - 1) / kBlocksPerShard;
  const long base = (long)shard * shard_cap;
  *b0 = base + min(n, (long)part * per);
  *b1 = base + min(n, (long)(part + 1) * per);
}

__global__ __launch_bounds__(kBinThreads) void k_dep_count(const uint32_t* __restrict__ key,
                                                           const unsigned long long* count, long shard_cap,
                                                           int n_rows, BinScratch bs) {
  __shared__ uint32_t lh[kMaxBinRows];
  for (int r = threadIdx.x; r < n_rows; r += blockDim.x) lh[r] = 0;
  __syncthreads();
  long b0, b1;
  block_range(count, shard_cap, &b0, &b1);
  for (long i = b0 + threadIdx.x; i < b1; i += blockDim.x) atomicAdd(&lh[key[i] >> kDepBinBits], 1u);
  __syncthreads();
  for (int r = threadIdx.x; r < n_rows; r += blockDim.x) bs.hist[(long)r * kBinBlocks + blockIdx.x] = lh[r];
}

// Block per row: exclusive prefix of the row's block counts (in place) and
// the row total.
__global__ __launch_bounds__(kBinBlocks) void k_dep_colscan(BinScratch bs) {
  __shared__ uint32_t v[kBinBlocks];
  const int r = blockIdx.x;
  uint32_t* h = bs.hist + (long)r * kBinBlocks;
  const uint32_t c = h[threadIdx.x];
  v[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < kBinBlocks; off <<= 1) {   // inclusive Hillis-Steele scan
    const uint32_t x = threadIdx.x >= (unsigned)off ? v[threadIdx.x - off] : 0u;
    __syncthreads();
    v[threadIdx.x] += x;
    __syncthreads();
  }
  h[threadIdx.x] = v[threadIdx.x] - c;
  if (threadIdx.x == kBinBlocks - 1) bs.total[r] = v[threadIdx.x];
}

// Exclusive scan of the row totals (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_dep_rowscan(int n_rows, BinScratch bs) {
  __shared__ uint32_t part[1024];
  const int per = (n_rows + 1023) / 1024;
  const int r0 = min(n_rows, (int)threadIdx.x * per), r1 = min(n_rows, r0 + per);
  uint32_t s = 0;
  for (int r = r0; r < r1; ++r) s += bs.total[r];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int r = r0; r < r1; ++r) {
    bs.row_begin[r] = run;
    run += bs.total[r];
  }
  if (threadIdx.x == 1023) bs.row_begin[n_rows] = part[1023];
}

// Records move in chunks of kScatChunk: each chunk is counted and ranked per
// row in LDS, the counts are scanned into staging offsets, the records are
// staged in row order with their final position in the spare word, and then
// written out by consecutive threads, so that a row's run of the chunk leaves
// as contiguous 16-byte stores instead of scattered ones.
constexpr int kScatChunk = 4 * kBinThreads;
constexpr int kRowsPerThread = kMaxBinRows / kBinThreads;
static_assert(kMaxBinRows % kBinThreads == 0, "rows per thread");

__global__ __launch_bounds__(kBinThreads) void k_dep_scatter(DepositList dep, const unsigned long long* count,
                                                             long shard_cap, int n_rows, BinScratch bs,
                                                             uint4* __restrict__ sorted) {
  __shared__ uint32_t cur[kMaxBinRows];   // next position of each row in this block's range
  __shared__ uint32_t off[kMaxBinRows];   // the chunk's count, then staging start, per row
  __shared__ uint4 stage[kScatChunk];
  __shared__ uint32_t wsum[kBinThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int r = tid; r < n_rows; r += blockDim.x)
    cur[r] = bs.row_begin[r] + bs.hist[(long)r * kBinBlocks + blockIdx.x];
  long b0, b1;
  block_range(count, shard_cap, &b0, &b1);
  const int R = (n_rows + kBinThreads - 1) / kBinThreads;   // rows owned per thread (<= kRowsPerThread)
  for (long c0 = b0; c0 < b1; c0 += kScatChunk) {
    const int nc = (int)min((long)kScatChunk, b1 - c0);
    for (int r = tid; r < n_rows; r += blockDim.x) off[r] = 0u;
    __syncthreads();
    uint32_t key[4], rank[4];
    float2 w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = u * kBinThreads + tid;
      if (j < nc) {
        key[u] = dep.key[c0 + j];
        w[u] = dep.w[c0 + j];
        rank[u] = atomicAdd(&off[key[u] >> kDepBinBits], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of the counts over the rows (thread t owns rows t R ..)
    uint32_t c[kRowsPerThread];
    uint32_t tsum = 0;
#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
      const int r = tid * R + j;
      c[j] = (j < R && r < n_rows) ? off[r] : 0u;
      tsum += c[j];
    }
    uint32_t incl = tsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (tid == 0) {
      uint32_t run = 0;
      for (int v = 0; v < kBinThreads / 64; ++v) {
        const uint32_t x = wsum[v];
        wsum[v] = run;
        run += x;
      }
    }
    __syncthreads();
    uint32_t at = wsum[wave] + incl - tsum;
#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
      const int r = tid * R + j;
      if (j < R && r < n_rows) { off[r] = at; at += c[j]; }
    }
    __syncthreads();
    // stage in row order, the final position in the spare word
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u * kBinThreads + tid < nc) {
        const uint32_t row = key[u] >> kDepBinBits;
        stage[off[row] + rank[u]] = make_uint4(key[u], __float_as_uint(w[u].x), __float_as_uint(w[u].y),
                                               cur[row] + rank[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
      const int r = tid * R + j;
      if (j < R && r < n_rows) cur[r] += c[j];
    }
    for (int j = tid; j < nc; j += kBinThreads) {
      const uint4 v = stage[j];
      sorted[v.w] = make_uint4(v.x, v.y, v.z, 0u);
    }
    __syncthreads();
  }
}

// Block (row, tile): the row's deposits summed into an LDS tile of samples
// [t0, t0 + kAccTile) in fixed-point units (integer LDS atomics), then added
// to h.
__global__ __launch_bounds__(512) void k_dep_accumulate(const uint4* __restrict__ sorted, BinScratch bs, uint32_t row0,
                                                        int n_t, int tiles, long long* __restrict__ h,
                                                        double scale, unsigned long long* over) {
  __shared__ unsigned long long acc[kAccTile];
  const int r = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const uint32_t i0 = bs.row_begin[r], i1 = bs.row_begin[r + 1];
  if (i0 == i1) return;   // nothing to add
  const int t0 = tile * kAccTile, len = min(kAccTile, n_t - t0);
  for (int j = threadIdx.x; j < len; j += blockDim.x) acc[j] = 0ull;
  __syncthreads();
  const uint32_t mask = (1u << kDepBinBits) - 1u;
  for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const uint4 rec = sorted[i];
    const int j0 = (int)(rec.x & mask) - 1;   // bin of w0; w1 goes to j0 + 1
    const int j = j0 - t0;
    if (j0 >= 0 && j >= 0 && j < len)
      atomicAdd(&acc[j], (unsigned long long)hist_units(__uint_as_float(rec.y), scale, over));
    if (j0 + 1 < n_t && j + 1 >= 0 && j + 1 < len)
      atomicAdd(&acc[j + 1], (unsigned long long)hist_units(__uint_as_float(rec.z), scale, over));
  }
  __syncthreads();
  long long* out = h + (long)(row0 + r) * n_t + t0;
  for (int j = threadIdx.x; j < len; j += blockDim.x) {
    const long long v = (long long)acc[j];
    if (v != 0) out[j] += v;
  }
}

// Block per RF row (n_t <= kAccTile, 1024 threads): the row of h (the
// deposits added directly) and the row's binned deposits summed in LDS in
// fixed-point units, then read out as fp32 into the same LDS and filtered
// with the pulse straight into rf: the histogram row never returns to HBM.
constexpr int kFuseThreads = 1024;
static_assert(kFuseThreads * kPulseR >= kAccTile, "one row per block");

template <bool kVec>
__global__ __launch_bounds__(kFuseThreads) void k_splat_pulse(const uint4* __restrict__ sorted, BinScratch bs,
                                                              uint32_t row0, int n_t, const long long* __restrict__ h,
                                                              double scale, unsigned long long* over,
                                                              const float* __restrict__ taps, int M,
                                                              float* __restrict__ rf) {
  __shared__ __align__(16) unsigned long long acc[kAccTile];   // then the fp32 input of the filter
  __shared__ __align__(16) float c[2 * kMaxTaps];
  __shared__ int row_over;
  const int r = blockIdx.x;
  const long grow = (long)row0 + r;
  const long long* hr = h + grow * n_t;
  for (int j = threadIdx.x; j < n_t; j += blockDim.x) acc[j] = (unsigned long long)hr[j];
  const int T = 2 * M + 1, Tp = fir_padded(M);
  for (int j = threadIdx.x; j < Tp; j += blockDim.x) c[j] = j < T ? taps[2 * M - j] : 0.0f;
  if (threadIdx.x == 0) row_over = 0;
  __syncthreads();
  const uint32_t i0 = bs.row_begin[r], i1 = bs.row_begin[r + 1];
  const uint32_t mask = (1u << kDepBinBits) - 1u;
  for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const uint4 rec = sorted[i];
    const int j0 = (int)(rec.x & mask) - 1;   // bin of w0; w1 goes to j0 + 1
    if (j0 >= 0) atomicAdd(&acc[j0], (unsigned long long)hist_units(__uint_as_float(rec.y), scale, over));
    if (j0 + 1 < n_t) atomicAdd(&acc[j0 + 1], (unsigned long long)hist_units(__uint_as_float(rec.z), scale, over));
  }
  __syncthreads();
  // read out: every thread takes its samples into registers before the fp32
  // copy (x[m] = h[m - M], zero outside [0, n_t)) overwrites the LDS
  constexpr int kPer = kAccTile / kFuseThreads;
  const double inv = 1.0 / scale;
  const bool bad = *over != 0ull;
  float v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int j = u * kFuseThreads + threadIdx.x;
    v[u] = j < n_t ? (bad ? __builtin_nanf("") : (float)((double)(long long)acc[j] * inv)) : 0.0f;
  }
  __syncthreads();
  float* x = reinterpret_cast<float*>(acc);
  const int n_x = kFuseThreads * kPulseR + Tp;   // every input the filter reads
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int j = u * kFuseThreads + threadIdx.x;
    if (j < n_t) x[M + j] = v[u];
  }
  for (int j = threadIdx.x; j < n_x; j += blockDim.x)
    if (j < M || j >= M + n_t) x[j] = 0.0f;
  __syncthreads();
  const int b = threadIdx.x * kPulseR;
  if (b < n_t) {
    float out[kPulseR];
    fir_block(x, c, b, Tp, out);
    fir_store<kVec>(rf + grow * n_t, b, n_t, out);
  }
}

}  // namespace

size_t splat_scratch_bytes(int n_rows) {
  return align256((size_t)kBinBlocks * n_rows * sizeof(uint32_t)) + align256((size_t)n_rows * sizeof(uint32_t)) +
         align256((size_t)(n_rows + 1) * sizeof(uint32_t));
}

void launch_splat_bin(const DepositList& dep, const unsigned long long* shard_count, long shard_cap,
                      int n_rows, uint4* sorted, void* scratch, hipStream_t s) {
  const BinScratch bs = carve(scratch, n_rows);
  hipLaunchKernelGGL(k_dep_count, dim3(kBinBlocks), dim3(kBinThreads), 0, s, dep.key, shard_count, shard_cap,
                     n_rows, bs);
  hipLaunchKernelGGL(k_dep_colscan, dim3(n_rows), dim3(kBinBlocks), 0, s, bs);
  hipLaunchKernelGGL(k_dep_rowscan, dim3(1), dim3(1024), 0, s, n_rows, bs);
  hipLaunchKernelGGL(k_dep_scatter, dim3(kBinBlocks), dim3(kBinThreads), 0, s, dep, shard_count, shard_cap,
                     n_rows, bs, sorted);
}

int launch_splat_pulse(const uint4* sorted, const void* scratch, uint32_t row0, int n_rows, int n_t,
                       const long long* h, double hist_scale, unsigned long long* hist_over, const float* taps,
                       int M, float* rf, hipStream_t s) {
  if (n_t > kAccTile || M > kMaxTaps - 1 || kFuseThreads * kPulseR + fir_padded(M) > 2 * kAccTile) return -1;
  const BinScratch bs = carve(const_cast<void*>(scratch), n_rows);
  const bool vec = n_t % 4 == 0 && ((uintptr_t)rf & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(k_splat_pulse<true>, dim3((unsigned)n_rows), dim3(kFuseThreads), 0, s, sorted, bs, row0, n_t,
                       h, hist_scale, hist_over, taps, M, rf);
  else
    hipLaunchKernelGGL(k_splat_pulse<false>, dim3((unsigned)n_rows), dim3(kFuseThreads), 0, s, sorted, bs, row0,
                       n_t, h, hist_scale, hist_over, taps, M, rf);
  return 0;
}

void launch_splat_accumulate(const uint4* sorted, const void* scratch, uint32_t row0, int n_rows,
                             int n_t, long long* h, double hist_scale, unsigned long long* hist_over,
                             hipStream_t s) {
  const BinScratch bs = carve(const_cast<void*>(scratch), n_rows);
  const int tiles = (n_t + kAccTile - 1) / kAccTile;
  hipLaunchKernelGGL(k_dep_accumulate, dim3((unsigned)((long)n_rows * tiles)), dim3(512), 0, s, sorted, bs,
                     row0, n_t, tiles, h, hist_scale, hist_over);
}

}  // namespace usrt
