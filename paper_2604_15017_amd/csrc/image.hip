// Image formation on gfx950 (paper Sec. 2.3.4 and Sec. 3.3): analytic signal
// of every RF channel (FFT in LDS), plane-wave delay-and-sum (Eq. das),
// envelope and log compression, and the adjoints of all three (Eq.
// das_adjoint as a per-sample gather, no atomics).
#include <algorithm>

#include "fir.h"
#include "kernels.h"

namespace usrt {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

constexpr int kFftThreads = 256;
constexpr int kMaxFft = 8192;
constexpr int kFftLoBits = 7;   // two-level twiddle table: 128 low and up to 64 high entries

// LDS index of element i: one float2 of padding every 16, so that the
// stride-R writes of the first pass spread over the banks.
__device__ __forceinline__ int fpad(int i) { return i + (i >> 4); }

constexpr int brev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}
constexpr int log2_c(int r) { return r <= 1 ? 0 : 1 + log2_c(r >> 1); }

// w_n^e = exp(-2 pi i e / n), 0 <= e < n, as hi[e >> 7] * lo[e & 127].
__device__ __forceinline__ float2 twid(const float2* lo, const float2* hi, int e) {
  return cmul(hi[e >> kFftLoBits], lo[e & ((1 << kFftLoBits) - 1)]);
}

// In-register R-point DFT, b_s = sum_r a_r w_R^(r s): radix-2 DIT on the
// bit-reversed registers, natural order out; w[t] = w_R^t, t < R / 2.
template <int R>
__device__ __forceinline__ void dft_regs(float2 (&a)[R], const float2 (&w)[R / 2 > 0 ? R / 2 : 1]) {
  constexpr int kLog = log2_c(R);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = brev_c(i, kLog);
    if (i < j) {
      const float2 t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
#pragma unroll
  for (int half = 1; half < R; half <<= 1)
#pragma unroll
    for (int base = 0; base < R; base += 2 * half)
#pragma unroll
      for (int q = 0; q < half; ++q) {
        const float2 t = q == 0 ? a[base + half] : cmul(a[base + q + half], w[q * (R / (2 * half))]);
        const float2 u = a[base + q];
        a[base + q] = cadd(u, t);
        a[base + q + half] = csub(u, t);
      }
}

enum FftIo : int {
  kIoLds,          // LDS buffer (padded)
  kIoRealPairIn,   // two global real rows as one complex row (row 0 + i row 1)
  kIoImagPairIn,   // the imaginary parts of two global complex rows, likewise
  kIoLdsQ,         // LDS, times the Hilbert multiplier -i sgn(k), conjugated
  kIoAnalyticOut,  // two global complex rows: (input row, its Hilbert transform)
  kIoAdjointOut    // two real rows (global or LDS): Re(input row) - Hilbert transform of its Im
};

// The two rows of one transform: row 0 at in / out, row 1 n elements after
// in and out_stride after out when two (else row 1 reads as zeros and is
// not written).
struct FftRows {
  const void* in;
  void* out;
  long out_stride;
  bool two;
};

// One Stockham radix-R pass (decimation in time, natural order in and out)
// over n points with L = product of the previous radices: butterfly j takes
// x[j + r n / R], twists it by w_(L R)^(r k), k = j mod L, transforms and
// writes y[(j / L) L R + k + s L]. Every thread first loads all its
// butterflies, so the pass can run in place in LDS.
template <int R, int kSrc, int kDst>
__device__ __forceinline__ void fft_pass(float2* x, const FftRows& io, int n, int L, const float2* lo,
                                         const float2* hi) {
  constexpr int kB = 32 / R > 0 ? 32 / R : 1;   // butterflies per thread (n <= 8192, 256 threads)
  const int m = n / R, Ls = L * R, tw_step = n / Ls;
  float2 a[kB][R];
  const int n1 = io.two ? n : 0;   // row 1, or row 0 again (read, then replaced by zeros)
#pragma unroll
  for (int bi = 0; bi < kB; ++bi) {
    const int j = threadIdx.x + bi * kFftThreads;
    if (j < m) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = j + r * m;
        if (kSrc == kIoRealPairIn) {
          const float* g = (const float*)io.in;
          const float v1 = g[n1 + i];
          a[bi][r] = make_float2(g[i], io.two ? v1 : 0.0f);
        } else if (kSrc == kIoImagPairIn) {
          const float2* g = (const float2*)io.in;
          const float v1 = g[n1 + i].y;
          a[bi][r] = make_float2(g[i].y, io.two ? v1 : 0.0f);
        } else {
          a[bi][r] = x[fpad(i)];
        }
      }
    }
  }
  if (kSrc == kIoLds) __syncthreads();   // every read before the in-place writes
  float2 w[R / 2 > 0 ? R / 2 : 1];
#pragma unroll
  for (int t = 0; t < R / 2; ++t) w[t] = twid(lo, hi, t * (n / R));
  const float inv_n = 1.0f / (float)n;
#pragma unroll
  for (int bi = 0; bi < kB; ++bi) {
    const int j = threadIdx.x + bi * kFftThreads;
    if (j < m) {
      const int k = j & (L - 1);
      if (L > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) a[bi][r] = cmul(a[bi][r], twid(lo, hi, r * k * tw_step));
      }
      dft_regs<R>(a[bi], w);
      const int base = (j - k) * R + k;
      if (kDst == kIoLds || kDst == kIoLdsQ) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int o = base + s * L;
          const float2 v = a[bi][s];
          if (kDst == kIoLds) {
            x[fpad(o)] = v;
          } else {
            // conj(-i sgn(o) v), sgn zero at o = 0 and o = n / 2
            const float sg = (o == 0 || o == (n >> 1)) ? 0.0f : (o < (n >> 1) ? 1.0f : -1.0f);
            x[fpad(o)] = make_float2(sg * v.y, sg * v.x);
          }
        }
      } else {
        // v = n conj(y) for y = Hilbert(row 0) + i Hilbert(row 1). The rows'
        // own samples at the outputs are read eight at a time ahead of the
        // stores (row 0 again in place of a missing row 1), so that a
        // group's loads are in flight together.
        constexpr int kG = R < 8 ? R : 8;
#pragma unroll
        for (int s0 = 0; s0 < R; s0 += kG) {
          float g0[kG], g1[kG];
#pragma unroll
          for (int t = 0; t < kG; ++t) {
            const int o = base + (s0 + t) * L;
            if (kDst == kIoAnalyticOut) {
              g0[t] = ((const float*)io.in)[o];
              g1[t] = ((const float*)io.in)[n1 + o];
            } else {
              g0[t] = ((const float2*)io.in)[o].x;
              g1[t] = ((const float2*)io.in)[n1 + o].x;
            }
          }
#pragma unroll
          for (int t = 0; t < kG; ++t) {
            const int o = base + (s0 + t) * L;
            const float2 v = a[bi][s0 + t];
            const float h0 = v.x * inv_n, h1 = -v.y * inv_n;
            if (kDst == kIoAnalyticOut) {
              float2* A = (float2*)io.out;
              A[o] = make_float2(g0[t], h0);
              if (io.two) A[io.out_stride + o] = make_float2(g1[t], h1);
            } else {
              float* gr = (float*)io.out;
              gr[o] = g0[t] - h0;
              if (io.two) gr[io.out_stride + o] = g1[t] - h1;
            }
          }
        }
      }
    }
  }
  if (kDst == kIoLds || kDst == kIoLdsQ) __syncthreads();
}

template <int kSrc, int kDst>
__device__ __forceinline__ void fft_pass_bits(int bits, float2* x, const FftRows& io, int n, int L,
                                              const float2* lo, const float2* hi) {
  switch (bits) {   // 64 <= n <= 8192 split into two or three passes: 3 to 5 bits each
    case 3: fft_pass<8, kSrc, kDst>(x, io, n, L, lo, hi); break;
    case 4: fft_pass<16, kSrc, kDst>(x, io, n, L, lo, hi); break;
    default: fft_pass<32, kSrc, kDst>(x, io, n, L, lo, hi); break;
  }
}

// The twiddle table w_n^e (two levels: lo[e & 127], hi[e >> 7]) in LDS from
// the first half kept on the device (w_n^(e + n/2) = -w_n^e), and the pass
// split of n = 2^logn: two or three passes of 3 to 5 bits, smallest first.
__device__ __forceinline__ int fft_setup(float2* lds, const float2* twiddle, int n, int logn, int bits[3]) {
  const int half = n >> 1;
  for (int i = threadIdx.x; i < (1 << kFftLoBits) + 64; i += blockDim.x) {
    const bool is_lo = i < (1 << kFftLoBits);
    const int e = is_lo ? i : (i - (1 << kFftLoBits)) << kFftLoBits;
    float2 v = make_float2(1.0f, 0.0f);
    if (e < n) {
      v = twiddle[e < half ? e : e - half];
      if (e >= half) v = make_float2(-v.x, -v.y);
    }
    lds[i] = v;
  }
  __syncthreads();
  const int n_pass = (logn + 4) / 5;
  for (int p = 0, left = logn; p < n_pass; ++p) {   // even split, smallest first
    bits[p] = left / (n_pass - p);
    left -= bits[p];
  }
  return n_pass;
}

// The Hilbert transforms of the two rows of io (the multiplier -i sgn(k),
// zero at k = 0 and n / 2): one complex transform of row 0 + i row 1, the
// multiplier, and the inverse taken as a forward transform of the conjugate;
// the last pass writes kOut.
template <int kIn, int kOut>
__device__ __forceinline__ void hilbert_pair(float2* x, const FftRows& io, int n, int n_pass, const int bits[3],
                                             const float2* lo, const float2* hi) {
  int L = 1;
  fft_pass_bits<kIn, kIoLds>(bits[0], x, io, n, L, lo, hi);
  L <<= bits[0];
  if (n_pass == 3) {
    fft_pass_bits<kIoLds, kIoLds>(bits[1], x, io, n, L, lo, hi);
    L <<= bits[1];
  }
  fft_pass_bits<kIoLds, kIoLdsQ>(bits[n_pass - 1], x, io, n, L, lo, hi);
  L = 1;
  for (int p = 0; p < n_pass - 1; ++p) {
    fft_pass_bits<kIoLds, kIoLds>(bits[p], x, io, n, L, lo, hi);
    L <<= bits[p];
  }
  // the last pass reads all of x before it writes (a barrier in between)
  fft_pass_bits<kIoLds, kOut>(bits[n_pass - 1], x, io, n, L, lo, hi);
}

// Analytic-signal map along the rows, T = F^-1 diag(H) F with H = 1, 2..2,
// 1, 0..0, written as A = x + i Hilbert(x) (H = 1 + sgn): the real part is
// the row itself and the imaginary part its Hilbert transform, two rows per
// block through one complex transform (the Hilbert transform is real, so it
// maps row 0 + i row 1 to the two transforms). Adjoint (kAdjoint): the map
// is real-linear from x to (Re A, Im A) and the Hilbert transform is
// antisymmetric, so g_rf = Re(g_A) - Hilbert(Im g_A). Block b takes rows 2b
// and 2b + 1 of n_rows.
template <bool kAdjoint>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_analytic(
    const void* in, void* out, const float2* twiddle, int n, int logn, long n_rows) {
  extern __shared__ float2 lds[];
  float2* lo = lds;                          // w_n^i, i < 128
  float2* hi = lds + (1 << kFftLoBits);       // w_n^(128 i), i < 64
  float2* x = hi + 64;
  int bits[3];
  const int n_pass = fft_setup(lds, twiddle, n, logn, bits);
  const long r0 = 2 * (long)blockIdx.x;
  const FftRows io{kAdjoint ? (const void*)((const float2*)in + r0 * n) : (const void*)((const float*)in + r0 * n),
                   kAdjoint ? (void*)((float*)out + r0 * n) : (void*)((float2*)out + r0 * n), (long)n,
                   r0 + 1 < n_rows};
  if (kAdjoint) hilbert_pair<kIoImagPairIn, kIoAdjointOut>(x, io, n, n_pass, bits, lo, hi);
  else hilbert_pair<kIoRealPairIn, kIoAnalyticOut>(x, io, n, n_pass, bits, lo, hi);
}

template <int R>
__device__ __forceinline__ void fir_row(const float* rr, const float* c, int Tp, int n, float* out) {
  for (int b = threadIdx.x * R; b < n; b += blockDim.x * R) {
    float acc[R];
    fir_block<R>(rr, c, b, Tp, acc);
    fir_store<true, R>(out, b, n, acc);
  }
}

// Row stride of the fused pulse adjoint's two real rows in LDS: the row, M
// zeros before it and Tp - M after it, rounded to four floats.
__host__ __device__ __forceinline__ int fir_row_stride(int n, int Tp) { return (n + Tp + 3) & ~3; }

// Adjoint of the pulse (Eq. axial_sig) after the adjoint of the analytic
// map, for rows 2b and 2b + 1: the transforms of k_analytic<true>, whose last
// pass writes the rows' real gradients into LDS (over the transform's
// buffer, M zeros before each and Tp - M after) instead of HBM, then the
// pulse correlation of k_pulse from each row (taps c[q] = taps[2M - q], the
// same fir_block sums), written as g_h. One HBM round trip of the rows less
// than the two kernels, and the same arithmetic in the same order.
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_analytic_pulse_adjoint(
    const float2* __restrict__ gA, float* __restrict__ gh, const float2* __restrict__ twiddle,
    const float* __restrict__ taps, int M, int n, int logn, long n_rows) {
  extern __shared__ float2 lds[];
  float2* lo = lds;
  float2* hi = lds + (1 << kFftLoBits);
  float2* x = hi + 64;
  int bits[3];
  const int n_pass = fft_setup(lds, twiddle, n, logn, bits);
  const long r0 = 2 * (long)blockIdx.x;
  const bool two = r0 + 1 < n_rows;
  const int T = 2 * M + 1, Tp = fir_padded(M), stride = fir_row_stride(n, Tp);
  float* rr = reinterpret_cast<float*>(x);   // rr[M + k], rr[stride + M + k]: sample k of the two rows
  const FftRows io{gA + r0 * n, rr + M, (long)stride, two};
  hilbert_pair<kIoImagPairIn, kIoAdjointOut>(x, io, n, n_pass, bits, lo, hi);
  float* c = rr + 2 * stride;
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    rr[j] = 0.0f;
    rr[stride + j] = 0.0f;
  }
  for (int j = M + n + threadIdx.x; j < n + Tp; j += blockDim.x) {
    rr[j] = 0.0f;
    rr[stride + j] = 0.0f;
  }
  for (int j = threadIdx.x; j < Tp; j += blockDim.x) c[j] = j < T ? taps[2 * M - j] : 0.0f;
  __syncthreads();
  fir_row<kPulseR>(rr, c, Tp, n, gh + r0 * (long)n);
  if (two) fir_row<kPulseR>(rr + stride, c, Tp, n, gh + (r0 + 1) * (long)n);
}

// Delay-and-sum, one pixel per thread, threads along z, reading the two
// samples of every (element, transmit) pair straight from HBM through the
// caches; used for grids too small to fill the chip with pixel tiles. The
// fractional sample index is formed in fp64 (an fp32 index near 4000 carries
// 2.4e-4 samples of rounding, i.e. 2e-4 rad of phase per tap at 5 MHz /
// 40 MHz); interpolation and accumulation are fp32, in the element-major pair
// order of the plain sum.
__global__ __launch_bounds__(256) void k_das_gather(const float2* __restrict__ A, float2* __restrict__ iq,
                                                    ProbeView p, GridView g, TxTable tx, int n_tx,
                                                    int tx_base, int accumulate) {
  const long px = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (px >= (long)g.n_x * g.n_z) return;
  const int a = (int)(px / g.n_z), b = (int)(px % g.n_z);
  const double x = g.x0 + a * g.dx, z = g.z0 + b * g.dz;
  const double s_per_m = p.fs / p.c_ref;
  float2 acc = accumulate ? iq[px] : make_float2(0.0f, 0.0f);
  const double half = 0.5 * (double)(p.n_elem - 1);
  for (int e = 0; e < p.n_elem; ++e) {
    const double dxe = x - ((double)e - half) * p.pitch;
    const double krx = sqrt(dxe * dxe + z * z) * s_per_m;
    for (int i = 0; i < n_tx; ++i) {
      const double k = (x * tx.sin_a[i] + z * tx.cos_a[i]) * s_per_m + krx;
      const double k0d = floor(k);
      if (!(k0d >= -1.0 && k0d < (double)p.n_t)) continue;
      const int k0 = (int)k0d;
      const float f = (float)(k - k0d);
      const float2* row = A + ((long)(tx_base + i) * p.n_elem + e) * p.n_t;
      const float2 v0 = k0 >= 0 ? row[k0] : make_float2(0.0f, 0.0f);
      const float2 v1 = k0 + 1 < p.n_t ? row[k0 + 1] : make_float2(0.0f, 0.0f);
      acc.x += (1.0f - f) * v0.x + f * v1.x;
      acc.y += (1.0f - f) * v0.y + f * v1.y;
    }
  }
  iq[px] = acc;
}

// One block per tile of kDasTx x kDasTz pixels, the (element, transmit) pairs
// taken element-major like the plain sum, kDasGroup at a time, in a two-stage
// pipeline: while the pixels interpolate group g from LDS, each thread holds
// its share of group g + 1's sample windows in registers (loads in flight),
// and the window bounds of group g + 2 are formed; one barrier per group.
// A pair's window is the range of samples any pixel of the tile can touch:
// the transmit term is linear in x and z, the receive distance lies between
// the distance from the element to the tile and to its farthest corner
// (fp64, one sample of slack on each side). A window wider than kDasSpan is
// read from HBM instead.
//
// Sample index: fs (x sin th + z cos th + r) / c_ref near 4000 needs more than
// fp32 (2.4e-4 samples of rounding, 2e-4 rad of phase at 5 MHz / 40 MHz), but
// only a few terms need fp64: the transmit term at the tile origin and the
// receive term per (pixel, element) are formed in fp64 and split into an
// integer and an fp32 fraction; the transmit term's change across the tile
// (at most tens of samples) is added in fp32. The index is then off by a few
// 1e-6 samples at most, and each pair costs fp32 and integer work only.
constexpr int kDasTx = 16, kDasTz = 16;      // 256 threads, z fastest
constexpr int kDasThreads = kDasTx * kDasTz;
constexpr int kDasGroup = 16;                // pairs per pipeline stage
constexpr int kDasBatch = 8;                 // pairs whose samples are read together
constexpr int kDasSpan = 144;                // window samples per pair in LDS (four blocks per CU)
constexpr int kDasStage = kDasGroup * kDasSpan / kDasThreads;   // staged samples per thread
static_assert(kDasGroup * kDasSpan % kDasThreads == 0, "window stage must split evenly");
static_assert(kDasGroup <= kDasThreads && kMaxTxPerLaunch <= kDasThreads, "one thread per bound");
constexpr long kDasMinTiles = 64;            // below this the grid cannot fill the chip: gather
constexpr long kDasSliceTiles = 1024;        // below this a tile's pairs are split over two slices

struct DasWindow { long row; int lo, n; };   // channel offset in A, first sample, length
struct TxSplit { int ib; float fb, da, db; };   // transmit term at the tile origin, steps per pixel

__device__ __forceinline__ DasWindow das_window(const ProbeView& p, const TxTable& tx, int n_tx, int tx_base,
                                                int q, double xa, double xb, double za, double zb) {
  const double s_per_m = p.fs / p.c_ref;
  const int e = q / n_tx, i = q % n_tx;
  const double xe = ((double)e - 0.5 * (double)(p.n_elem - 1)) * p.pitch;
  const double sa = tx.sin_a[i], ca = tx.cos_a[i];
  const double l1 = xa * sa + za * ca, l2 = xb * sa + za * ca, l3 = xa * sa + zb * ca, l4 = xb * sa + zb * ca;
  const double lmin = fmin(fmin(l1, l2), fmin(l3, l4)), lmax = fmax(fmax(l1, l2), fmax(l3, l4));
  const double dx_near = xe < xa ? xa - xe : (xe > xb ? xe - xb : 0.0);
  const double dx_far = fmax(fabs(xe - xa), fabs(xe - xb));
  const double rmin = sqrt(dx_near * dx_near + za * za), rmax = sqrt(dx_far * dx_far + zb * zb);
  // samples [klo, khi], not clipped to the record: the loader fills samples
  // outside [0, n_t) with zeros, so a tap reads its two samples from the
  // window and taps beyond the record add zero, as the plain sum skips them
  // (the limits below only keep far-off windows finite; they come out wide)
  const double klo = floor((lmin + rmin) * s_per_m) - 1.0, khi = floor((lmax + rmax) * s_per_m) + 2.0;
  const double lo = fmax(klo, -2.0 * kDasSpan), hi = fmin(khi, (double)p.n_t + 2.0 * kDasSpan);
  return DasWindow{((long)(tx_base + i) * p.n_elem + e) * p.n_t, (int)lo, hi >= lo ? (int)(hi - lo) + 1 : 0};
}

// Tile order: the chip deals consecutive blocks round-robin to its kXcds
// XCDs, each with its own L2. Block b runs tile L = (b % kXcds) per_xcd +
// b / kXcds of the x-fastest tile order, so each XCD owns a contiguous band
// of depths and the tiles it runs at one time are x-neighbours at the same
// depths, which read nearly the same sample windows of every pair: the
// windows come from HBM about once and are shared in that XCD's L2.
constexpr int kXcds = 8;

template <int kS>
__global__ __launch_bounds__(kDasThreads * kS) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_das_tiled(const float2* __restrict__ A, float2* __restrict__ iq, ProbeView p, GridView g, TxTable tx,
                 int n_tx, int tx_base, int accumulate, int tiles_x, int tiles_z) {
  __shared__ float2 win[kS][2][kDasGroup * kDasSpan];
  __shared__ DasWindow wb[kS][3][kDasGroup];
  __shared__ int wide[kS][3];   // the group is partial or has a window wider than kDasSpan or under 2
  __shared__ TxSplit ts[kMaxTxPerLaunch];
  // kS slices of kDasThreads threads share the tile: slice sl takes the
  // sl-th run of pair groups, and the partial sums are added in slice order
  // the slice is uniform over each wave (kDasThreads is a multiple of 64), so
  // the pair bookkeeping below stays in scalar registers
  const int sl = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kDasThreads);
  const int tid = (int)threadIdx.x % kDasThreads;
  const int n_tiles = tiles_x * tiles_z, per_xcd = (n_tiles + kXcds - 1) / kXcds;
  const int tile = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (tile >= n_tiles) return;   // the whole block: the last band is short
  const int a0 = (tile % tiles_x) * kDasTx, b0 = (tile / tiles_x) * kDasTz;
  const int ia = tid / kDasTz, ib = tid % kDasTz;
  const int a = a0 + ia, b = b0 + ib;
  const bool inside = a < g.n_x && b < g.n_z;
  const long px = (long)a * g.n_z + b;
  const double x = g.x0 + a * g.dx, z = g.z0 + b * g.dz;
  // the tile's extent (clipped to the grid)
  const double xa = g.x0 + a0 * g.dx, xb = g.x0 + (min(a0 + kDasTx, g.n_x) - 1) * g.dx;
  const double za = g.z0 + b0 * g.dz, zb = g.z0 + (min(b0 + kDasTz, g.n_z) - 1) * g.dz;
  const double s_per_m = p.fs / p.c_ref;
  const double half = 0.5 * (double)(p.n_elem - 1);
  const int n_pairs = p.n_elem * n_tx;
  const int n_groups = (n_pairs + kDasGroup - 1) / kDasGroup;
  // groups per slice (the same loop count for all), first group, end of pairs
  const int per = kS == 1 ? n_groups : (n_groups + kS - 1) / kS;
  const int g0 = kS == 1 ? 0 : sl * per;
  const int q_end = kS == 1 ? n_pairs : min(n_pairs, (g0 + per) * kDasGroup);
  if ((int)threadIdx.x < n_tx) {
    const int i = threadIdx.x;
    const double kt = (xa * tx.sin_a[i] + za * tx.cos_a[i]) * s_per_m;
    const double fl = floor(kt);
    ts[i] = TxSplit{(int)fl, (float)(kt - fl), (float)(g.dx * tx.sin_a[i] * s_per_m),
                    (float)(g.dz * tx.cos_a[i] * s_per_m)};
  }
  auto bounds = [&](int grp, int buf) {   // grp: the slice's own group index
    const int q = (g0 + grp) * kDasGroup + tid;
    if (tid < kDasGroup) {
      const DasWindow w = q < q_end ? das_window(p, tx, n_tx, tx_base, q, xa, xb, za, zb) : DasWindow{0, 0, 0};
      wb[sl][buf][tid] = w;
      const unsigned long long m = __ballot(q >= q_end || w.n > kDasSpan || w.n < 2);   // the slice's lanes 0..15
      if (tid == 0) wide[sl][buf] = m != 0ull;
    }
  };
  float2 st[kDasStage];
  auto load = [&](const DasWindow* w) {
#pragma unroll
    for (int r = 0; r < kDasStage; ++r) {
      const int f = r * kDasThreads + tid;
      const int j = f / kDasSpan, t = f - j * kDasSpan;
      const DasWindow ww = w[j];
      const int k = ww.lo + t;
      st[r] = (t < ww.n && ww.n <= kDasSpan && k >= 0 && k < p.n_t) ? A[ww.row + k] : make_float2(0.0f, 0.0f);
    }
  };
  auto store = [&](float2* dst) {
#pragma unroll
    for (int r = 0; r < kDasStage; ++r) dst[r * kDasThreads + tid] = st[r];
  };

  bounds(0, 0);
  if (per > 1) bounds(1, 1);
  __syncthreads();
  load(wb[sl][0]);
  store(win[sl][0]);
  __syncthreads();

  float2 acc = (accumulate && inside && sl == 0) ? iq[px] : make_float2(0.0f, 0.0f);
  const float fa = (float)ia, fz = (float)ib;
  const int q_first = min(g0 * kDasGroup, n_pairs);
  int e = q_first / n_tx, i = q_first % n_tx, rx_e = -1, rx_i = 0;
  float rx_f = 0.0f;
  for (int grp = 0; grp < per; ++grp) {
    const int cur = grp & 1;
    const DasWindow* wc = wb[sl][grp % 3];
    if (grp + 1 < per) load(wb[sl][(grp + 1) % 3]);          // in flight during the sums below
    if (grp + 2 < per) bounds(grp + 2, (grp + 2) % 3);
    const int nq = min(kDasGroup, q_end - (g0 + grp) * kDasGroup);
    const float2* wcur = win[sl][cur];
    if (!wide[sl][grp % 3]) {
      // whole group, every window in LDS: all indices first, then the reads
      // and sums without branches (samples outside the record are zeros)
#pragma unroll 1
      for (int j0 = 0; j0 < kDasGroup; j0 += kDasBatch) {
        int kk[kDasBatch];
        float fk[kDasBatch];
#pragma unroll
        for (int j = 0; j < kDasBatch; ++j) {
          if (e != rx_e) {
            const double dxe = x - ((double)e - half) * p.pitch;
            const double krx = sqrt(dxe * dxe + z * z) * s_per_m;
            const double fl = floor(krx);
            rx_i = (int)fl;
            rx_f = (float)(krx - fl);
            rx_e = e;
          }
          const TxSplit T = ts[i];
          const float sf = (T.fb + rx_f) + fmaf(fa, T.da, fz * T.db);
          const float fl = floorf(sf);
          kk[j] = T.ib + rx_i + (int)fl;
          fk[j] = sf - fl;
          if (++i == n_tx) { i = 0; ++e; }
        }
#pragma unroll
        for (int j = 0; j < kDasBatch; ++j) {
          const DasWindow w = wc[j0 + j];
          // within [0, n - 2] by the window bound (n >= 2 in this path);
          // clamped so that a read never leaves the pair's window
          const int o = (j0 + j) * kDasSpan + min(max(kk[j] - w.lo, 0), w.n - 2);
          const float2 v0 = wcur[o], v1 = wcur[o + 1];
          acc.x += fmaf(fk[j], v1.x - v0.x, v0.x);
          acc.y += fmaf(fk[j], v1.y - v0.y, v0.y);
        }
      }
    } else for (int j = 0; j < nq; ++j) {
      if (inside) {
        if (e != rx_e) {   // receive term once per element: integer + fraction
          const double dxe = x - ((double)e - half) * p.pitch;
          const double krx = sqrt(dxe * dxe + z * z) * s_per_m;
          const double fl = floor(krx);
          rx_i = (int)fl;
          rx_f = (float)(krx - fl);
          rx_e = e;
        }
        const TxSplit T = ts[i];
        const float sf = (T.fb + rx_f) + fmaf(fa, T.da, fz * T.db);
        const float fl = floorf(sf);
        const int k0 = T.ib + rx_i + (int)fl;
        const float f = sf - fl;
        const DasWindow w = wc[j];
        if (k0 >= -1 && k0 < p.n_t && w.n >= 2) {
          float2 v0, v1;
          if (w.n <= kDasSpan) {
            const int o = min(max(k0 - w.lo, 0), w.n - 2);   // within [0, n - 2] by the window bound
            v0 = wcur[j * kDasSpan + o];
            v1 = wcur[j * kDasSpan + o + 1];
          } else {
            const float2* row = A + w.row;
            v0 = k0 >= 0 ? row[k0] : make_float2(0.0f, 0.0f);
            v1 = k0 + 1 < p.n_t ? row[k0 + 1] : make_float2(0.0f, 0.0f);
          }
          acc.x += (1.0f - f) * v0.x + f * v1.x;
          acc.y += (1.0f - f) * v0.y + f * v1.y;
        }
      }
      if (++i == n_tx) { i = 0; ++e; }
    }
    if (grp + 1 < per) store(win[sl][cur ^ 1]);
    __syncthreads();
  }
  if (kS > 1) {   // slice partial sums, added in slice order (the loop ended with a barrier)
    float2* part = &win[0][0][0];
    if (sl > 0) part[(sl - 1) * kDasThreads + tid] = acc;
    __syncthreads();
    if (sl == 0) {
      for (int t = 1; t < kS; ++t) {
        const float2 v = part[(t - 1) * kDasThreads + tid];
        acc.x += v.x;
        acc.y += v.y;
      }
      if (inside) iq[px] = acc;
    }
  } else if (inside) {
    iq[px] = acc;
  }
}

// Frame maximum of |I|^2 with the first index among equals, packed as
// (float bits << 32) | (~index) for a 64-bit atomic max.
__global__ __launch_bounds__(256) void k_env_max(const float2* __restrict__ iq, long n,
                                                 unsigned long long* key) {
  __shared__ unsigned long long best;
  if (threadIdx.x == 0) best = 0;
  __syncthreads();
  unsigned long long local = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 v = iq[i];
    const float pw = v.x * v.x + v.y * v.y;
    const unsigned long long kk = ((unsigned long long)__float_as_uint(pw) << 32) |
                                  (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
    local = kk > local ? kk : local;
  }
  atomicMax(&best, local);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(key, best);
}

__device__ __forceinline__ float key_power(unsigned long long key) {
  return __uint_as_float((unsigned)(key >> 32));
}
__device__ __forceinline__ long key_index(unsigned long long key) {
  return (long)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFu));
}

constexpr float kLog10Scale = 10.0f;                 // 20 log10 |I| = 10 log10 |I|^2
constexpr double kDbPerNeper = 8.685889638065037;    // 20 / ln 10

__global__ __launch_bounds__(256) void k_bmode(const float2* __restrict__ iq, long n, float dr,
                                               const unsigned long long* key, float* out) {
  const float m2 = key_power(*key);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 v = iq[i];
    const float pw = v.x * v.x + v.y * v.y;
    float b = pw > 0.0f ? kLog10Scale * log10f(pw / m2) : -dr;
    out[i] = fmaxf(b, -dr);
  }
}

// Sum of the block's per-thread values in a fixed tree (256 threads).
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// g_I = g_B (20/ln10) I / |I|^2 on unclipped pixels; the sum of g_B over
// them (block sums added to the order-independent accumulator sum[kSumWords])
// feeds the normalisation term added at the arg-max pixel afterwards.
__global__ __launch_bounds__(256) void k_bmode_vjp(const float2* __restrict__ iq,
                                                   const float* __restrict__ gb, long n, float dr,
                                                   const unsigned long long* key, unsigned long long* sum,
                                                   float2* __restrict__ giq) {
  const float m2 = key_power(*key);
  double local = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 v = iq[i];
    const float pw = v.x * v.x + v.y * v.y;
    const bool live = pw > 0.0f && kLog10Scale * log10f(pw / m2) > -dr;
    float2 gi = make_float2(0.0f, 0.0f);
    if (live) {
      const float s = gb[i] * (float)kDbPerNeper / pw;
      gi = make_float2(s * v.x, s * v.y);
      local += gb[i];
    }
    giq[i] = gi;
  }
  const double bs = block_sum256(local);
  if (threadIdx.x == 0) sum_add(sum, bs);
}

__global__ void k_bmode_vjp_fix(const float2* __restrict__ iq, const unsigned long long* key,
                                const unsigned long long* sum, float2* giq) {
  const long am = key_index(*key);
  const float m2 = key_power(*key);
  const float2 v = iq[am];
  const float s = (float)(-kDbPerNeper * sum_value(sum) / (double)m2);
  giq[am].x += s * v.x;
  giq[am].y += s * v.y;
}

// Adjoint of DAS for one RF row (transmit, element): each thread owns kS
// consecutive samples k and gathers, column by column, the pixels whose
// interpolation reads them with weight max(0, 1 - |kappa - k|). kappa(z) is
// increasing in z, so the first pixel of interest follows from the inverse
// z(kappa) = (T^2 - dx^2) / (T cos th + sqrt(T^2 - dx^2 sin^2 th)),
// T = kappa c / fs - x sin th; weights are recomputed exactly per pixel, so
// rounding in the inverse only shifts where the walk starts.
template <int kS>
__global__ __launch_bounds__(256) void k_das_adjoint(const float2* __restrict__ giq,
                                                     float2* __restrict__ gA, ProbeView p,
                                                     GridView g, TxTable tx, int tx_base) {
  const int txl = blockIdx.x / p.n_elem;
  const int e = blockIdx.x % p.n_elem;
  const int k_a = threadIdx.x * kS;
  // this thread's kS accumulators, private, interleaved across the block's
  // threads (entry s at acc[s * blockDim.x]): a pixel adds to two of them
  extern __shared__ float2 acc_lds[];
  float2* acc = acc_lds + threadIdx.x;
  const int step = blockDim.x;
  for (int s = 0; s < kS; ++s) acc[s * step] = make_float2(0.0f, 0.0f);
  const double sa = tx.sin_a[txl], ca = tx.cos_a[txl];
  const double s_per_m = p.fs / p.c_ref, m_per_s = p.c_ref / p.fs;
  const double xe = ((double)e - 0.5 * (double)(p.n_elem - 1)) * p.pitch;
  if (k_a < p.n_t) {
    for (int a = 0; a < g.n_x; ++a) {
      const double x = g.x0 + a * g.dx;
      const double dx = x - xe;
      // first pixel with kappa > k_a - 1
      const double T = (double)(k_a - 1) * m_per_s - x * sa;
      const double disc = T * T - dx * dx * sa * sa;
      int b = 0;
      if (T > 0.0 && disc >= 0.0) {
        const double zs = (T * T - dx * dx) / (T * ca + sqrt(disc));
        const double bd = floor((zs - g.z0) / g.dz) - 1.0;
        b = bd > 0.0 ? (bd < (double)g.n_z ? (int)bd : g.n_z) : 0;
      }
      const float2* col = giq + (long)a * g.n_z;
      for (; b < g.n_z; ++b) {
        const double z = g.z0 + b * g.dz;
        const double kap = (x * sa + z * ca + sqrt(dx * dx + z * z)) * s_per_m;
        if (kap >= (double)(k_a + kS)) break;
        const double rel = kap - (double)k_a;
        if (rel <= -1.0) continue;
        const float2 gv = col[b];
        // the forward reads sample floor(kap) with weight 1 - f and the next with f
        const double j0d = floor(rel);
        const int j0 = (int)j0d;
        const float f = (float)(rel - j0d);
        if (j0 >= 0) {
          float2 v = acc[j0 * step];
          v.x = fmaf(1.0f - f, gv.x, v.x);
          v.y = fmaf(1.0f - f, gv.y, v.y);
          acc[j0 * step] = v;
        }
        if (j0 + 1 < kS) {
          float2 v = acc[(j0 + 1) * step];
          v.x = fmaf(f, gv.x, v.x);
          v.y = fmaf(f, gv.y, v.y);
          acc[(j0 + 1) * step] = v;
        }
      }
    }
    float2* row = gA + ((long)(tx_base + txl) * p.n_elem + e) * p.n_t;
    for (int s = 0; s < kS; ++s)
      if (k_a + s < p.n_t) row[k_a + s] = acc[s * step];
  }
}

// Square root of s to about 1e-14 relative: the fp32 root refined by one
// Newton step whose residual s - r0^2 is formed in fp64 (a handful of
// instructions against the fp64 root's iteration).
__device__ __forceinline__ double sqrt_newton(double s) {
  if (!(s > 1e-30)) return sqrt(s);
  const float r0 = __builtin_amdgcn_sqrtf((float)s);
  const double r0d = (double)r0;
  return r0d + (double)((float)fma(-r0d, r0d, s) * (0.5f * __builtin_amdgcn_rcpf(r0)));
}

// Adjoint of DAS for kT RF rows of one element (kT transmits), column by
// column: the block's threads take the pixels of one column (coalesced reads
// of dL/dI, the next column's prefetched into registers while this one is
// summed) and add each pixel's two tent weights into the rows' accumulators
// in LDS. The receive distance of a pixel is formed once for the kT rows.
// Down a column kappa grows by more than two samples per pixel (checked by
// the launcher: dz fs / c_ref cos(theta) > 2 and z0 >= 0), so the pixels of
// one column touch disjoint sample pairs of a row and need no atomics; a
// barrier separates the columns. Every sample then sums its contributions in
// column order, as the per-sample gather does.
constexpr int kAdjThreads = 512;
constexpr int kAdjMaxR = 4;   // pixels per thread and column: n_z <= 2048

template <int kT>
__global__ __launch_bounds__(kAdjThreads) void k_das_adjoint_cols(const float2* __restrict__ giq,
                                                                  float2* __restrict__ gA, ProbeView p,
                                                                  GridView g, TxTable tx, int n_tx,
                                                                  int tx_base) {
  const int groups = (n_tx + kT - 1) / kT;
  const int e = blockIdx.x / groups, i0 = (blockIdx.x % groups) * kT;
  const int nt = min(kT, n_tx - i0);
  extern __shared__ float2 acc_row[];   // [kT][n_t]
  for (int k = threadIdx.x; k < kT * p.n_t; k += blockDim.x) acc_row[k] = make_float2(0.0f, 0.0f);
  __syncthreads();
  double sa[kT], ca[kT];
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    const int i = i0 + min(t, nt - 1);
    sa[t] = tx.sin_a[i];
    ca[t] = tx.cos_a[i];
  }
  const double s_per_m = p.fs / p.c_ref;
  const double xe = ((double)e - 0.5 * (double)(p.n_elem - 1)) * p.pitch;
  float2 cur[kAdjMaxR], nxt[kAdjMaxR];
  auto fetch = [&](int a, float2* v) {
    const float2* col = giq + (long)a * g.n_z;
#pragma unroll
    for (int r = 0; r < kAdjMaxR; ++r) {
      const int b = (int)threadIdx.x + r * kAdjThreads;
      v[r] = b < g.n_z ? col[b] : make_float2(0.0f, 0.0f);
    }
  };
  fetch(0, cur);
  for (int a = 0; a < g.n_x; ++a) {
    if (a + 1 < g.n_x) fetch(a + 1, nxt);
    const double x = g.x0 + a * g.dx;
    const double dx = x - xe;
#pragma unroll
    for (int r = 0; r < kAdjMaxR; ++r) {
      const int b = (int)threadIdx.x + r * kAdjThreads;
      if (b >= g.n_z) continue;
      const double z = g.z0 + b * g.dz;
      const double rx = sqrt_newton(dx * dx + z * z);
      const float2 gv = cur[r];
#pragma unroll
      for (int t = 0; t < kT; ++t) {
        if (t >= nt) continue;
        float2* acc = acc_row + t * p.n_t;
        const double kap = (x * sa[t] + z * ca[t] + rx) * s_per_m;
        const double k0d = floor(kap);
        if (!(k0d >= -1.0 && k0d < (double)p.n_t)) continue;
        const int k0 = (int)k0d;
        const float f = (float)(kap - k0d);
        if (k0 >= 0) {
          float2 v = acc[k0];
          v.x = fmaf(1.0f - f, gv.x, v.x);
          v.y = fmaf(1.0f - f, gv.y, v.y);
          acc[k0] = v;
        }
        if (k0 + 1 < p.n_t) {
          float2 v = acc[k0 + 1];
          v.x = fmaf(f, gv.x, v.x);
          v.y = fmaf(f, gv.y, v.y);
          acc[k0 + 1] = v;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kAdjMaxR; ++r) cur[r] = nxt[r];
  }
  for (int t = 0; t < nt; ++t) {
    float2* row = gA + ((long)(tx_base + i0 + t) * p.n_elem + e) * p.n_t;
    for (int k = threadIdx.x; k < p.n_t; k += blockDim.x) row[k] = acc_row[t * p.n_t + k];
  }
}

// Gradients of Re<g, I> with respect to the acquisition parameters of Eq.
// das (the steering angle of each transmit, c_ref, the pitch) at fixed
// analytic signal. I depends on them only through the fractional sample index
// k = fs tau, and the interpolation's slope in k is A[k0 + 1] - A[k0]; with
// k = fs ((x sin th + z cos th) + r_e) / c_ref and x_e = (e - (N - 1)/2) pitch:
// dk/dth = fs (x cos th - z sin th) / c_ref, dk/dc_ref = -k / c_ref,
// dk/dpitch = -fs (x - x_e) (e - (N - 1)/2) / (r_e c_ref). Block (tile of
// kAcqThreads pixels, transmit): each thread sums over the elements for its
// pixel in fp64, the block reduces its three sums in a fixed order into one
// partial row per tile.
constexpr int kAcqThreads = 256;

__global__ __launch_bounds__(kAcqThreads) void k_das_acq(const float2* __restrict__ A,
                                                         const float2* __restrict__ giq, ProbeView p,
                                                         GridView g, TxTable tx, int tx_base,
                                                         double* __restrict__ part) {
  __shared__ double red[3][kAcqThreads];
  const int i = blockIdx.y, tid = threadIdx.x;
  const long n_px = (long)g.n_x * g.n_z;
  const long px = (long)blockIdx.x * kAcqThreads + tid;
  double s_th = 0.0, s_c = 0.0, s_p = 0.0;
  if (px < n_px) {
    const int a = (int)(px / g.n_z), b = (int)(px % g.n_z);
    const double x = g.x0 + a * g.dx, z = g.z0 + b * g.dz;
    const double s_per_m = p.fs / p.c_ref;
    const double sa = tx.sin_a[i], ca = tx.cos_a[i];
    const double kt = (x * sa + z * ca) * s_per_m;
    const double dk_dth = (x * ca - z * sa) * s_per_m;
    const double half = 0.5 * (double)(p.n_elem - 1);
    const float2 gv = giq[px];
    const float2* rows = A + (long)(tx_base + i) * p.n_elem * p.n_t;
    for (int e = 0; e < p.n_elem; ++e) {
      const double de = (double)e - half;
      const double dxe = x - de * p.pitch;
      const double r = sqrt(dxe * dxe + z * z);
      const double k = kt + r * s_per_m;
      const double k0d = floor(k);
      if (!(k0d >= -1.0 && k0d < (double)p.n_t)) continue;
      const int k0 = (int)k0d;
      const float2* row = rows + (long)e * p.n_t;
      const float2 v0 = k0 >= 0 ? row[k0] : make_float2(0.0f, 0.0f);
      const float2 v1 = k0 + 1 < p.n_t ? row[k0 + 1] : make_float2(0.0f, 0.0f);
      const double dl = (double)gv.x * ((double)v1.x - (double)v0.x) + (double)gv.y * ((double)v1.y - (double)v0.y);
      s_th += dl * dk_dth;
      s_c -= dl * k;
      s_p -= dl * dxe * de / r;
    }
    s_c /= p.c_ref;
    s_p *= s_per_m;
  }
  red[0][tid] = s_th;
  red[1][tid] = s_c;
  red[2][tid] = s_p;
  __syncthreads();
  for (int off = kAcqThreads / 2; off > 0; off >>= 1) {
    if (tid < off) {
      red[0][tid] += red[0][tid + off];
      red[1][tid] += red[1][tid + off];
      red[2][tid] += red[2][tid + off];
    }
    __syncthreads();
  }
  if (tid < 3) part[((long)i * gridDim.x + blockIdx.x) * 3 + tid] = red[tid][0];
}

// Block j adds, in a fixed order, the partial rows of output j of one launch
// group into out: j < n_tx the angle of transmit tx_base + j, then c_ref and
// the pitch (summed over the group's transmits too).
__global__ __launch_bounds__(256) void k_acq_reduce(const double* __restrict__ part, int n_tx, int n_tiles,
                                                    int tx_base, int n_tx_total, double* __restrict__ out) {
  __shared__ double red[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  double v = 0.0;
  if (j < n_tx) {
    for (int t = tid; t < n_tiles; t += 256) v += part[((long)j * n_tiles + t) * 3];
  } else {
    const int c = j - n_tx + 1;
    for (long q = tid; q < (long)n_tx * n_tiles; q += 256) v += part[q * 3 + c];
  }
  red[tid] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) out[j < n_tx ? tx_base + j : n_tx_total + (j - n_tx)] += red[0];
}

// L = (1/n) sum [l1 |d| + l2 d^2], d = B - R; dL/dB = (l1 sign(d) + 2 l2 d) / n.
// Block sums go into the order-independent accumulator acc[kSumWords];
// k_loss_finish writes the total.
__global__ __launch_bounds__(256) void k_image_loss(const float* __restrict__ b,
                                                    const float* __restrict__ ref, long n,
                                                    double l1, double l2, unsigned long long* acc,
                                                    float* __restrict__ gb) {
  const double inv_n = 1.0 / (double)n;
  double local = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double d = (double)b[i] - (double)ref[i];
    local += l1 * fabs(d) + l2 * d * d;
    if (gb) {
      const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
      gb[i] = (float)((l1 * sg + 2.0 * l2 * d) * inv_n);
    }
  }
  const double bs = block_sum256(local);
  if (threadIdx.x == 0) sum_add(acc, bs * inv_n);
}

__global__ void k_loss_finish(const unsigned long long* acc, double* loss) { *loss = sum_value(acc); }

int grid_for(long n, int per_block, int cap) {
  long gsz = (n + per_block - 1) / per_block;
  if (gsz < 1) gsz = 1;
  return (int)(gsz < cap ? gsz : cap);
}

int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

}  // namespace

size_t analytic_lds(int n_t) {
  return (size_t)((1 << kFftLoBits) + 64 + n_t + n_t / 16 + 1) * sizeof(float2);
}

int launch_analytic(const float* rf, float2* A, const float2* twiddle, int n_t, long n_rows,
                    hipStream_t s) {
  const int logn = log2_exact(n_t);
  if (logn < 6 || n_t > kMaxFft) return -1;
  const size_t lds = analytic_lds(n_t);
  hipLaunchKernelGGL(k_analytic<false>, dim3((unsigned)((n_rows + 1) / 2)), dim3(kFftThreads), lds, s,
                     (const void*)rf, (void*)A, twiddle, n_t, logn, n_rows);
  return 0;
}

int launch_analytic_adjoint(const float2* g_A, float* g_rf, const float2* twiddle, int n_t,
                            long n_rows, hipStream_t s) {
  const int logn = log2_exact(n_t);
  if (logn < 6 || n_t > kMaxFft) return -1;
  const size_t lds = analytic_lds(n_t);
  hipLaunchKernelGGL(k_analytic<true>, dim3((unsigned)((n_rows + 1) / 2)), dim3(kFftThreads), lds, s,
                     (const void*)g_A, (void*)g_rf, twiddle, n_t, logn, n_rows);
  return 0;
}

int launch_analytic_pulse_adjoint(const float2* g_A, float* g_h, const float2* twiddle, const float* taps_reversed,
                                  int M, int n_t, long n_rows, hipStream_t s) {
  const int logn = log2_exact(n_t);
  if (logn < 6 || n_t > kMaxFft || M < 0 || M > kMaxTaps - 1) return -1;
  // the transform's buffer, or the two padded real rows and the taps after the twiddles
  const int Tp = fir_padded(M);
  const size_t fir = (size_t)((1 << kFftLoBits) + 64) * sizeof(float2) +
                     (size_t)(2 * fir_row_stride(n_t, Tp) + Tp) * sizeof(float);
  const size_t lds = std::max(analytic_lds(n_t), fir);
  hipLaunchKernelGGL(k_analytic_pulse_adjoint, dim3((unsigned)((n_rows + 1) / 2)), dim3(kFftThreads), lds, s, g_A,
                     g_h, twiddle, taps_reversed, M, n_t, logn, n_rows);
  return 0;
}

void launch_das(const float2* A, float2* iq, const ProbeView& p, const GridView& g,
                const TxTable& tx, int n_tx_group, int tx_base, bool accumulate, hipStream_t s) {
  const int tiles_x = (g.n_x + kDasTx - 1) / kDasTx, tiles_z = (g.n_z + kDasTz - 1) / kDasTz;
  const long tiles = (long)tiles_x * tiles_z;
  if (tiles >= kDasMinTiles) {
    // grids of fewer than 1024 tiles split each tile's pairs over two slices
    // of one block, so that the chip still holds four waves per SIMD
    const unsigned blocks = (unsigned)(kXcds * ((tiles + kXcds - 1) / kXcds));
    if (tiles < kDasSliceTiles)
      hipLaunchKernelGGL(k_das_tiled<2>, dim3(blocks), dim3(2 * kDasThreads), 0, s, A, iq, p, g, tx,
                         n_tx_group, tx_base, accumulate ? 1 : 0, tiles_x, tiles_z);
    else
      hipLaunchKernelGGL(k_das_tiled<1>, dim3(blocks), dim3(kDasThreads), 0, s, A, iq, p, g, tx,
                         n_tx_group, tx_base, accumulate ? 1 : 0, tiles_x, tiles_z);
  } else {
    const long n_px = (long)g.n_x * g.n_z;
    hipLaunchKernelGGL(k_das_gather, dim3((unsigned)((n_px + 255) / 256)), dim3(256), 0, s, A, iq, p, g, tx,
                       n_tx_group, tx_base, accumulate ? 1 : 0);
  }
}

void launch_env_max(const float2* iq, long n_px, unsigned long long* key, hipStream_t s) {
  hipLaunchKernelGGL(k_env_max, dim3(grid_for(n_px, 256, 1024)), dim3(256), 0, s, iq, n_px, key);
}

void launch_bmode(const float2* iq, long n_px, float dr_db, const unsigned long long* key,
                  float* bmode, hipStream_t s) {
  hipLaunchKernelGGL(k_bmode, dim3(grid_for(n_px, 256, 4096)), dim3(256), 0, s, iq, n_px, dr_db,
                     key, bmode);
}

void launch_bmode_vjp(const float2* iq, const float* g_b, long n_px, float dr_db,
                      const unsigned long long* key, unsigned long long* sum, float2* g_iq, hipStream_t s) {
  hipLaunchKernelGGL(k_bmode_vjp, dim3(grid_for(n_px, 256, 1024)), dim3(256), 0, s, iq, g_b, n_px,
                     dr_db, key, sum, g_iq);
}

void launch_bmode_vjp_fix(const float2* iq, long n_px, const unsigned long long* key,
                          const unsigned long long* sum, float2* g_iq, hipStream_t s) {
  (void)n_px;
  hipLaunchKernelGGL(k_bmode_vjp_fix, dim3(1), dim3(1), 0, s, iq, key, sum, g_iq);
}

constexpr size_t kAdjLds = 64 * 1024;   // accumulator rows per column-kernel block

void launch_das_adjoint(const float2* g_iq, float2* g_A, const ProbeView& p, const GridView& g,
                        const TxTable& tx, int n_tx_group, int tx_base, hipStream_t s) {
  const dim3 grid((unsigned)(n_tx_group * p.n_elem)), block(256);
  // column kernel when a column's pixels cannot share a tent sample: kappa
  // grows by at least dz fs / c_ref cos(theta) per pixel for z >= 0
  double ca_min = 1.0;
  for (int i = 0; i < n_tx_group; ++i) ca_min = std::min(ca_min, tx.cos_a[i]);
  const bool cols_ok = g.z0 >= 0.0 && g.dz * p.fs / p.c_ref * ca_min > 2.0 + 1e-9 &&
                       g.n_z <= kAdjThreads * kAdjMaxR && (size_t)p.n_t * sizeof(float2) <= kAdjLds;
  if (cols_ok) {
    // as many transmits per block as the LDS budget holds
    const size_t row = (size_t)p.n_t * sizeof(float2);
    const int kt = 4 * row <= kAdjLds ? 4 : (2 * row <= kAdjLds ? 2 : 1);
    const int groups = (n_tx_group + kt - 1) / kt;
    const dim3 cgrid((unsigned)(groups * p.n_elem)), cblock(kAdjThreads);
    if (kt == 4)
      hipLaunchKernelGGL(k_das_adjoint_cols<4>, cgrid, cblock, 4 * row, s, g_iq, g_A, p, g, tx, n_tx_group, tx_base);
    else if (kt == 2)
      hipLaunchKernelGGL(k_das_adjoint_cols<2>, cgrid, cblock, 2 * row, s, g_iq, g_A, p, g, tx, n_tx_group, tx_base);
    else
      hipLaunchKernelGGL(k_das_adjoint_cols<1>, cgrid, cblock, row, s, g_iq, g_A, p, g, tx, n_tx_group, tx_base);
    return;
  }
  const int per_thread = (p.n_t + 255) / 256;
  const int k_s = per_thread <= 8 ? 8 : (per_thread <= 16 ? 16 : 32);
  const size_t lds = (size_t)k_s * 256 * sizeof(float2);   // 64 KB at most
  if (per_thread <= 8)
    hipLaunchKernelGGL(k_das_adjoint<8>, grid, block, lds, s, g_iq, g_A, p, g, tx, tx_base);
  else if (per_thread <= 16)
    hipLaunchKernelGGL(k_das_adjoint<16>, grid, block, lds, s, g_iq, g_A, p, g, tx, tx_base);
  else
    hipLaunchKernelGGL(k_das_adjoint<32>, grid, block, lds, s, g_iq, g_A, p, g, tx, tx_base);
}

long das_acq_tiles(const GridView& g) { return ((long)g.n_x * g.n_z + kAcqThreads - 1) / kAcqThreads; }

void launch_das_acq(const float2* A, const float2* g_iq, const ProbeView& p, const GridView& g, const TxTable& tx,
                    int n_tx_group, int tx_base, int n_tx_total, double* part, double* out, hipStream_t s) {
  const long tiles = das_acq_tiles(g);
  hipLaunchKernelGGL(k_das_acq, dim3((unsigned)tiles, (unsigned)n_tx_group), dim3(kAcqThreads), 0, s, A, g_iq,
                     p, g, tx, tx_base, part);
  hipLaunchKernelGGL(k_acq_reduce, dim3((unsigned)(n_tx_group + 2)), dim3(256), 0, s, part, n_tx_group,
                     (int)tiles, tx_base, n_tx_total, out);
}

int launch_pulse_adjoint(const float* g_rf, float* g_h, const float* taps_reversed, int M, int n_t,
                         long n_rows, hipStream_t s) {
  return launch_pulse(g_rf, g_h, taps_reversed, M, n_t, n_rows, s);
}

}  // namespace usrt

namespace usrt {
void launch_image_loss(const float* b, const float* ref, long n, double l1, double l2,
                       unsigned long long* acc, double* loss, float* gb, hipStream_t s) {
  hipLaunchKernelGGL(k_image_loss, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, b, ref, n, l1, l2,
                     acc, gb);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(1), 0, s, acc, loss);
}
}  // namespace usrt
