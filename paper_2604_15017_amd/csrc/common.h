// Device-side building blocks for the gfx950 kernels: counter-based RNG,
// fp64 3-vectors, scene/probe views and the per-ray decision hash.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace usrt {

constexpr int kMaxRegions = 64;
constexpr int kMaxPlanes = 16;
constexpr int kMaxSpheres = 32;
constexpr int kMaxTxPerLaunch = 64;
constexpr int kMaxMeshes = 32;
constexpr int kMaxCylinders = 16;
constexpr int kMaxBvhDepth = 38;        // levels of the binary tree the hierarchy is built as
constexpr int kMaxBvhStack = 60;        // LDS stack entries of the 4-wide walk: three per level
constexpr double kTMin = 1e-6;          // self-intersection guard [m]
// Outward padding of the hierarchy's fp32 boxes [m]: it covers the rounding of
// a ray's origin, inverse direction and slab distances to fp32 (a few nm at
// the scenes' scale), so the fp32 box tests never miss a box the fp64 ray enters.
constexpr float kBoxPad = 1e-6f;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11). key = (seed, 0),
// counter = (ray id, transmit id, event, 0). The 64x64 -> 128 products are
// formed from 32-bit halves by the compiler (__umul64hi).
// ---------------------------------------------------------------------------
struct U64x4 { uint64_t v[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = 0xD2E7470EE14C6C93ULL * c0;
    const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ULL, c0);
    const uint64_t lo1 = 0xCA5A826395121157ULL * c2;
    const uint64_t hi1 = __umul64hi(0xCA5A826395121157ULL, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B97F4A7C15ULL;
    k1 += 0xBB67AE8584CAA73BULL;
  }
  return U64x4{{c0, c1, c2, c3}};
}

// 23 random bits as the odd multiple (2 m + 1) 2^-24: exact in fp32 and fp64.
__device__ __forceinline__ double unit_uniform(uint64_t x) {
  return ((double)(x >> 41) + 0.5) * 0x1.0p-23;
}

struct Draw { double u0, u1, u2, u3; };

__device__ __forceinline__ Draw draw(uint64_t seed, uint32_t ray, uint32_t tx_id, uint32_t event) {
  const U64x4 o = philox4x64_10(ray, tx_id, event, 0, seed, 0);
  return Draw{unit_uniform(o.v[0]), unit_uniform(o.v[1]), unit_uniform(o.v[2]),
              unit_uniform(o.v[3])};
}

// Decision hash event: SplitMix64 finaliser of (tag, event index, word).
__device__ __forceinline__ uint64_t event_mix(uint32_t tag, uint32_t k, uint32_t word) {
  uint64_t z = ((uint64_t)tag << 60) | ((uint64_t)(k & 0xFFFu) << 48) | (uint64_t)word;
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
enum : uint32_t { kEvHit = 1, kEvArray = 2, kEvBranch = 3, kEvNee = 4 };
enum : int { kHitNone = 0, kHitPlane = 1, kHitSphere = 2, kHitArray = 3, kHitMesh = 4, kHitCylinder = 5 };

// Inner node of the 4-wide bounding-volume hierarchy (128 B): the fp32 boxes
// of up to four children (rounded outward), one coordinate per 16-byte row,
// and the child references. A reference c >= 0 is an inner node; c < 0 is a
// leaf holding the n = (~c) & 15 triangles starting at (~c) >> 4 in leaf
// order; an unused slot is the empty leaf ~0 with a point box far away.
struct alignas(16) BvhNode {
  float lox[4], loy[4], loz[4], hix[4], hiy[4], hiz[4];
  int child[4];
  int pad[4];
};
static_assert(sizeof(BvhNode) == 128, "hierarchy node layout");
constexpr int kEmptyChild = ~0;
constexpr float kFarBox = 1e30f;
constexpr int kLeafCap = 15;

// Leaf-order triangle as the walk reads it: p0 and the edges p1 - p0,
// p2 - p0 in fp64 (80 B, 16-B aligned), rewritten by every refit.
struct TriRec {
  double p0[3], e1[3], e2[3], pad;
};

// Read-only pointer into device memory in the global address space. The
// scene's array pointers live in the per-block LDS copy of the scene; typed
// this way, loads through them are global loads rather than flat ones (a flat
// load also counts against the LDS wait counter, so every wait on an LDS read
// of the walk's stack would wait for the node loads in flight as well).
template <class T> using gptr = __attribute__((address_space(1))) const T*;

// Whole-structure load through a gptr, as 16-byte vector loads.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ T gload(gptr<T> p) {
  static_assert(sizeof(T) % 16 == 0, "16-byte pieces");
  T out;
  const __attribute__((address_space(1))) u32x4* q = (const __attribute__((address_space(1))) u32x4*)p;
  u32x4* o = reinterpret_cast<u32x4*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 16); ++i) o[i] = q[i];
  return out;
}

struct d3 { double x, y, z; };
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator*(d3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Probe as the kernels see it.
struct ProbeView {
  int n_elem, n_t;
  double pitch, elem_w, elem_h, f0, fs, c_ref, alpha_m, alpha_c;
  double cos_m, cos_c;   // cos(alpha_m), cos(alpha_c)
};

// Scene as the kernels see it (device pointers; copied to LDS per block).
struct SceneView {
  const double* theta;
  const int* plane_regions;
  const double* plane_kd;
  const int* sphere_regions;
  const double* sphere_kd;
  int n_regions, n_planes, n_spheres, start_region;
  double np_per_m;       // amplitude attenuation [Np/m] per dB/cm/MHz at f0
  // cylinders along y: (x - cx)^2 + (z - cz)^2 = R^2
  int n_cylinders;
  const int* cylinder_regions;   // [n_cylinders][2]: inside, outside
  const double* cylinder_kd;
  // triangle meshes (all null / zero without meshes)
  int n_meshes, n_basis;
  int stack_cap;               // LDS stack entries per thread (3 per inner level)
  const int* mesh_regions;     // [n_meshes][2]: inside, outside
  const double* mesh_kd;       // [n_meshes]
  const BvhNode* nodes;
  const TriRec* trec;          // leaf order: current geometry
  const int4* tri;             // leaf order: vertex ids (x, y, z), mesh id (w)
  const int* tri_orig;         // leaf order -> triangle id of the description
  const double* vcur;          // [V][3] current vertex positions
  const double* vnormal;       // [V][3] displacement directions
  const double* vbasis;        // [V][n_basis]
};

// Per-block copy of the scene in LDS.
struct SceneLDS {
  double c[kMaxRegions], Z[kMaxRegions], a[kMaxRegions];
  double ic[kMaxRegions];   // 1 / c: travel time per metre
  double pd[kMaxPlanes], pkd[kMaxPlanes];
  int pr[kMaxPlanes][2];
  double sx[kMaxSpheres], sy[kMaxSpheres], sz[kMaxSpheres], sr[kMaxSpheres], skd[kMaxSpheres];
  int sreg[kMaxSpheres][2];
  int mreg[kMaxMeshes][2];
  double mkd[kMaxMeshes];
  double cx[kMaxCylinders], cz[kMaxCylinders], cr[kMaxCylinders], ckd[kMaxCylinders];
  int creg[kMaxCylinders][2];
  double prho[kMaxPlanes], srho[kMaxSpheres], crho[kMaxCylinders], mrho[kMaxMeshes];   // GGX roughness
  int n_planes, n_spheres, n_cylinders, n_meshes, start_region, stack_cap;
  bool any_diffuse;
  gptr<BvhNode> nodes;
  gptr<TriRec> trec;
  gptr<int4> tri;
  gptr<int> tri_orig;
  gptr<double> vcur;
};

__device__ inline void load_scene(SceneLDS& s, const SceneView& v) {
  const int t = threadIdx.x;
  const int nr = v.n_regions;
  for (int i = t; i < nr; i += blockDim.x) {
    s.c[i] = v.theta[3 * i];
    s.ic[i] = 1.0 / v.theta[3 * i];
    s.Z[i] = v.theta[3 * i + 1];
    s.a[i] = v.theta[3 * i + 2] * v.np_per_m;
  }
  const int op = 3 * nr, os = op + v.n_planes;
  for (int i = t; i < v.n_planes; i += blockDim.x) {
    s.pd[i] = v.theta[op + i];
    s.pkd[i] = v.plane_kd[i];
    s.pr[i][0] = v.plane_regions[2 * i];
    s.pr[i][1] = v.plane_regions[2 * i + 1];
  }
  for (int i = t; i < v.n_spheres; i += blockDim.x) {
    s.sx[i] = v.theta[os + 4 * i];
    s.sy[i] = v.theta[os + 4 * i + 1];
    s.sz[i] = v.theta[os + 4 * i + 2];
    s.sr[i] = v.theta[os + 4 * i + 3];
    s.skd[i] = v.sphere_kd[i];
    s.sreg[i][0] = v.sphere_regions[2 * i];
    s.sreg[i][1] = v.sphere_regions[2 * i + 1];
  }
  for (int i = t; i < v.n_meshes; i += blockDim.x) {
    s.mreg[i][0] = v.mesh_regions[2 * i];
    s.mreg[i][1] = v.mesh_regions[2 * i + 1];
    s.mkd[i] = v.mesh_kd[i];
  }
  const int oc = os + 4 * v.n_spheres;
  for (int i = t; i < v.n_cylinders; i += blockDim.x) {
    s.cx[i] = v.theta[oc + 3 * i];
    s.cz[i] = v.theta[oc + 3 * i + 1];
    s.cr[i] = v.theta[oc + 3 * i + 2];
    s.ckd[i] = v.cylinder_kd[i];
    s.creg[i][0] = v.cylinder_regions[2 * i];
    s.creg[i][1] = v.cylinder_regions[2 * i + 1];
  }
  // roughness follows the cylinders: planes, spheres, cylinders, meshes
  const int orh = oc + 3 * v.n_cylinders;
  const int n1 = v.n_planes, n2 = n1 + v.n_spheres, n3 = n2 + v.n_cylinders;
  for (int i = t; i < n3 + v.n_meshes; i += blockDim.x) {
    const double r = v.theta[orh + i];
    if (i < n1) s.prho[i] = r;
    else if (i < n2) s.srho[i - n1] = r;
    else if (i < n3) s.crho[i - n2] = r;
    else s.mrho[i - n3] = r;
  }
  if (t == 0) {
    s.n_planes = v.n_planes;
    s.n_spheres = v.n_spheres;
    s.n_cylinders = v.n_cylinders;
    s.n_meshes = v.n_meshes;
    s.stack_cap = v.stack_cap;
    s.start_region = v.start_region;
    bool d = false;
    for (int i = 0; i < v.n_planes; ++i) d |= v.plane_kd[i] > 0.0;
    for (int i = 0; i < v.n_spheres; ++i) d |= v.sphere_kd[i] > 0.0;
    for (int i = 0; i < v.n_cylinders; ++i) d |= v.cylinder_kd[i] > 0.0;
    for (int i = 0; i < v.n_meshes; ++i) d |= v.mesh_kd[i] > 0.0;
    s.any_diffuse = d;
    s.nodes = (gptr<BvhNode>)v.nodes;
    s.trec = (gptr<TriRec>)v.trec;
    s.tri = (gptr<int4>)v.tri;
    s.tri_orig = (gptr<int>)v.tri_orig;
    s.vcur = (gptr<double>)v.vcur;
  }
  __syncthreads();
}

// Transmit table passed by value.
struct TxTable {
  double sin_a[kMaxTxPerLaunch], cos_a[kMaxTxPerLaunch];
  uint32_t id[kMaxTxPerLaunch];
  int n;
};

// Receive directivity (Eq. cutoff) as a function of the cosine of the angle
// between the element normal and the direction the wave comes from: 1 up to
// alpha_m, 0 beyond alpha_c (both tested on the cosine), linear in the angle
// between.
// Out-of-line arc cosine, exponential, sine and cosine for the transport and
// replay loops: inlined, their polynomials' constants are hoisted out of the
// loops and spilled, and every ray reloads them from scratch memory.
struct SinCos { double s, c; };
__device__ __attribute__((noinline)) double exp_ool(double x) { return exp(x); }
__device__ __attribute__((noinline)) double acos_ool(double x) { return acos(x); }
__device__ __attribute__((noinline)) SinCos sincos_ool(double x) { return SinCos{sin(x), cos(x)}; }

// The ramp between the two angles, out of line: inlined, the arc cosine's
// constants were hoisted out of the transport loops and spilled, and every
// ray reloaded them.
__device__ __attribute__((noinline)) double rx_ramp(const ProbeView& p, double c) {
  return (p.alpha_c - acos(c)) / (p.alpha_c - p.alpha_m);
}
__device__ __forceinline__ double rx_directivity(const ProbeView& p, double cos_a) {
  const double c = fmin(1.0, fmax(-1.0, cos_a));
  if (c >= p.cos_m) return 1.0;
  if (c < p.cos_c) return 0.0;
  return rx_ramp(p, c);
}

// Block-level reduction of the event counters into the global int64[5]:
// primary segments, secondary segments, deposits, interactions, secondary
// rays. Called by every thread of the block (it contains barriers).
__device__ __forceinline__ void flush_counters(unsigned long long* g, unsigned long long c0,
                                               unsigned long long c1, unsigned long long c2,
                                               unsigned long long c3, unsigned long long c4) {
  __shared__ unsigned long long acc[5];
  if (threadIdx.x < 5) acc[threadIdx.x] = 0;
  __syncthreads();
  if (c0) atomicAdd(&acc[0], c0);
  if (c1) atomicAdd(&acc[1], c1);
  if (c2) atomicAdd(&acc[2], c2);
  if (c3) atomicAdd(&acc[3], c3);
  if (c4) atomicAdd(&acc[4], c4);
  __syncthreads();
  if (threadIdx.x < 5 && acc[threadIdx.x]) atomicAdd(&g[threadIdx.x], acc[threadIdx.x]);
}

// Block-aggregated append to two queues at once. Each lane with keep_a
// (keep_b) receives a distinct slot in queue A (B). The two running counts
// share one 64-bit word (A in the low half, B in the high half), so a block
// takes all its slots with a single atomic. Must be called by every thread of
// the block (it contains barriers); `scratch` is (waves per block) + 1 words
// of LDS.
struct Slots { long a, b; };

__device__ __forceinline__ Slots block_append2(bool keep_a, bool keep_b,
                                               unsigned long long* counts,
                                               unsigned long long* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
  const unsigned long long ma = __ballot(keep_a), mb = __ballot(keep_b);
  if (lane == 0) scratch[wave] = ((unsigned long long)__popcll(mb) << 32) | (unsigned)__popcll(ma);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int w = 0; w < n_waves; ++w) {   // exclusive scan over the waves
      const unsigned long long c = scratch[w];
      scratch[w] = run;
      run += c;
    }
    scratch[n_waves] = run ? atomicAdd(counts, run) : 0ull;
  }
  __syncthreads();
  const unsigned long long base = scratch[n_waves] + scratch[wave];
  __syncthreads();   // scratch is reused by the next call
  const unsigned below_a =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0u));
  const unsigned below_b =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
  Slots s;
  s.a = keep_a ? (long)(uint32_t)base + below_a : -1;
  s.b = keep_b ? (long)(base >> 32) + below_b : -1;
  return s;
}

// Block-aggregated append to one queue; same contract as block_append2.
__device__ __forceinline__ long block_append1(bool keep, unsigned long long* count,
                                              unsigned long long* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
  const unsigned long long m = __ballot(keep);
  if (lane == 0) scratch[wave] = (unsigned long long)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int w = 0; w < n_waves; ++w) {
      const unsigned long long c = scratch[w];
      scratch[w] = run;
      run += c;
    }
    scratch[n_waves] = run ? atomicAdd(count, run) : 0ull;
  }
  __syncthreads();
  const unsigned long long base = scratch[n_waves] + scratch[wave];
  __syncthreads();
  const unsigned below =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  return keep ? (long)(base + below) : -1;
}

// Appends one entry per active lane whose `want` is set, with one atomic per
// wave; usable in divergent code (only the active lanes take part).
__device__ __forceinline__ long wave_append(bool want, unsigned long long* count) {
  const unsigned long long m = __ballot(want);
  if (!want) return -1;
  const int leader = __ffsll((long long)m) - 1;
  const unsigned below =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  unsigned long long base = 0;
  if (below == 0) base = atomicAdd(count, (unsigned long long)__popcll(m));
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)base, leader);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
  return (long)((((unsigned long long)hi << 32) | lo) + below);
}

// One path contribution of amplitude a at time t on RF row `row`, split by
// the linear tent: a (1 - f) at bin j0 = floor(t fs), a f at j0 + 1 (bins
// outside [0, n_t) are dropped when the deposit is added).
struct Deposit {
  uint32_t row;
  int32_t j0;
  float w0, w1;
};

__device__ __forceinline__ bool make_deposit(uint32_t row, int n_t, double fs, double t, double a,
                                             Deposit* d) {
  const double x = t * fs;
  if (!(x > -1.0 && x < (double)n_t)) return false;   // also rejects NaN
  const double j0d = floor(x);
  const double f = x - j0d;
  d->row = row;
  d->j0 = (int)j0d;
  d->w0 = (float)(a * (1.0 - f));
  d->w1 = (float)(a * f);
  return true;
}

// ---------------------------------------------------------------------------
// Order-independent sums of fp64 values. A value v is cut at fixed binary
// boundaries: with its leading bit in window b (windows of 32 bits, window b
// holding multiples of 2^(32 b + kSumBase)), the integer pieces hi and lo of
// v / 2^(32 (b - 1) + kSumBase), truncated towards zero (at least 33
// significant bits kept), are added to the int64 words b and b - 1 of the
// accumulator. Integer addition is associative, so the total is the same
// whatever order the threads add in. Each word takes 2^31 pieces before it
// could overflow. Values below 2^(kSumBase + 32) are dropped; a value above
// the last window increments the overflow word, and the total then reads NaN.
// ---------------------------------------------------------------------------
constexpr int kSumBins = 10;                  // windows: 2^-168 .. 2^120
constexpr int kSumBase = -200;
constexpr int kSumWords = kSumBins + 1;       // the windows, then the overflow count

struct SumPieces { int b; unsigned long long hi, lo; bool over; };

__host__ __device__ __forceinline__ bool sum_pieces(double v, SumPieces* p) {
  if (v == 0.0) return false;
  const double a = fabs(v);
  int e;
  frexp(a, &e);                               // a in [2^(e-1), 2^e)
  const int b = (e - 1 - kSumBase) >> 5;      // window of the leading bit
  if (b < 1) return false;                    // below the first window: dropped
  if (!(b < kSumBins)) {                      // beyond the last window (or not finite)
    p->over = true;
    return true;
  }
  const double scaled = ldexp(a, -(32 * (b - 1) + kSumBase));   // in [2^32, 2^64)
  const unsigned long long u = (unsigned long long)scaled;
  unsigned long long hi = u >> 32, lo = u & 0xFFFFFFFFull;
  if (v < 0.0) { hi = 0ull - hi; lo = 0ull - lo; }
  p->b = b;
  p->hi = hi;
  p->lo = lo;
  p->over = false;
  return true;
}

// Adds v to an accumulator whose kSumWords words lie `stride` words apart,
// acc[w * stride] (LDS or global memory).
__device__ __forceinline__ void sum_add(unsigned long long* acc, long stride, double v) {
  SumPieces p;
  if (!sum_pieces(v, &p)) return;
  if (p.over) { atomicAdd(acc + kSumBins * stride, 1ull); return; }
  atomicAdd(acc + p.b * stride, p.hi);
  if (p.lo) atomicAdd(acc + (p.b - 1) * stride, p.lo);
}

// Adds v to the contiguous accumulator acc[kSumWords].
__device__ __forceinline__ void sum_add(unsigned long long* acc, double v) { sum_add(acc, 1, v); }

// The accumulated total: the windows added in a fixed order.
__host__ __device__ __forceinline__ double sum_value(const unsigned long long* acc) {
  if (acc[kSumBins]) return __builtin_nan("");
  double r = 0.0;
  for (int b = 0; b < kSumBins; ++b) {
    const long long w = (long long)acc[b];
    if (w) r += ldexp((double)w, 32 * b + kSumBase);
  }
  return r;
}

// Recorded deposits, structure of arrays: key = (row - row0) << kDepBinBits |
// (j0 + 1), w = (w0, w1).
constexpr int kDepBinBits = 19;
constexpr int kMaxBinRows = 8192;                          // rows of one binned group
constexpr int kMaxBinSamples = (1 << kDepBinBits) - 1;     // n_t below this
constexpr int kDepShards = 64;   // record buffer shards, each with its own counter
struct DepositList {
  uint32_t* key;
  float2* w;
  uint32_t row0;
};

// The deposit histogram is fixed point: a bin holds an int64 count of units
// of 1/scale, so that sums of deposits added by many threads in any order
// are the same integers. A tent weight is rounded to fp32 first and then to
// the nearest unit (the same rounding whether it is recorded for the binned
// splat or added at once). hist_scale puts the weight of one emitted ray,
// 1/rays_per_elem, at 2^40 units or more (a power of two, so the read-out
// divides exactly); a single weight beyond kHistMaxUnits units (2^12 and more
// emitted-ray weights) is clamped and counted in the overflow word, and the
// RF rows then read NaN.
constexpr double kHistMaxUnits = 4503599627370496.0;   // 2^52

inline double hist_scale(int rays_per_elem) {
  int e = 0;
  while ((1L << e) < (long)rays_per_elem) ++e;
  return ldexp(1.0, 40 + e);
}

__device__ __forceinline__ long long hist_units(float w, double scale, unsigned long long* over) {
  double x = (double)w * scale;
  if (!(fabs(x) <= kHistMaxUnits)) {   // also NaN
    atomicAdd(over, 1ull);
    x = x > 0.0 ? kHistMaxUnits : -kHistMaxUnits;
  }
  return (long long)rint(x);
}

// Adds a deposit straight into the histogram with global integer atomics.
__device__ __forceinline__ void add_deposit(long long* h, int n_t, const Deposit& d, double scale,
                                            unsigned long long* over) {
  unsigned long long* r = (unsigned long long*)(h + (long)d.row * n_t);
  if (d.j0 >= 0) atomicAdd(r + d.j0, (unsigned long long)hist_units(d.w0, scale, over));
  if (d.j0 + 1 < n_t) atomicAdd(r + d.j0 + 1, (unsigned long long)hist_units(d.w1, scale, over));
}

}  // namespace usrt
