// Forward Monte-Carlo transport for gfx950 (paper Sec. 2.3), wavefront style:
// one launch per interaction index k, each consuming a compacted queue of
// live rays in HBM and producing the next one, plus one launch per k for the
// receiver-directed secondary rays spawned at diffuse-capable hits. Deposits
// are splatted with a linear tent into a fixed-point histogram
// h[tx][elem][sample] (int64 units, integer atomics: the sums do not depend on
// the order of the additions); a final FIR applies the pulse of Eq. axial_sig.
//
// Precision: positions, directions, times and weights are fp64 (MI355X issues
// an fp64 FMA at the rate of an unpacked fp32 one). A time error dt costs
// 2 pi f0 dt of phase, and the parity bound on RF needs dt of a few ps over
// paths tens of millimetres long, which fp32 geometry cannot hold.
#include "kernels.h"
#include "fir.h"
#include "geometry.h"

namespace usrt {

// One interaction step for every live ray (k = 1 fuses the emission).
template <bool kAudit, bool kMeshes>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMeshes ? 4 : 3, 8))) void k_bounce(TraceArgs a, int k) {
  const long n_in = k == 1 ? a.n_chunk : (long)(uint32_t)a.counts[k - 1];
  if ((long)blockIdx.x * blockDim.x >= n_in) return;   // whole block idle
  __shared__ SceneLDS S;
  __shared__ unsigned long long scan[8];
  extern __shared__ int bvh_stack[];   // stack_cap entries per thread when the scene has meshes
  load_scene(S, a.scene);
  int* stk = bvh_stack + threadIdx.x;
  const ProbeView& P = a.probe;
  const long stride = (long)gridDim.x * blockDim.x;
  unsigned long long n_seg = 0, n_dep = 0, n_int = 0;

  // block-uniform loop: the queue append below synchronises the block
  for (long base = (long)blockIdx.x * blockDim.x; base < n_in; base += stride) {
    const long i = base + threadIdx.x;
    const bool active = i < n_in;
    d3 o{0, 0, 0}, d{0, 0, 1};
    double t = 0.0, w = 0.0;
    uint32_t rid = 0, meta = 0;
    if (active) {
      if (k == 1) {
        const long g = a.g0 + i;
        const int txl = (int)(g / a.ray_count);
        rid = (uint32_t)(a.ray_begin + g % a.ray_count);
        const int e = (int)(rid / (uint32_t)a.rays_per_elem);
        const Draw u = draw(a.seed, rid, a.tx.id[txl], 0);
        const double sa = a.tx.sin_a[txl], ca = a.tx.cos_a[txl];
        o = d3{elem_x(P, e) + (u.u0 - 0.5) * P.elem_w, (u.u1 - 0.5) * P.elem_h, 0.0};
        d = d3{sa, 0.0, ca};
        t = o.x * (sa / P.c_ref);
        w = fmax(0.0, ca) / (double)a.rays_per_elem;
        meta = (uint32_t)S.start_region | (1u << 8) | ((uint32_t)txl << 12);
      } else {
        o = d3{a.qin.ox[i], a.qin.oy[i], a.qin.oz[i]};
        d = d3{a.qin.dx[i], a.qin.dy[i], a.qin.dz[i]};
        t = a.qin.t[i];
        w = a.qin.w[i];
        rid = a.qin.rid[i];
        meta = a.qin.meta[i];
      }
    }
    int region = meta & 0xFF;
    bool delta = (meta >> 8) & 1u;
    const int txl = (int)(meta >> 12);
    bool keep = false, push_nee = false;
    d3 x{0, 0, 0};
    double nee_amp = 0.0;
    int nee_e = 0;
    const int incident_region = region;   // the secondary ray starts in this medium
    uint64_t hsum = 0;

    if (active) {
      const Hit h = closest_hit<kMeshes>(S, o, d, true, stk);
      ++n_seg;
      if (kAudit) hsum += event_mix(kEvHit, k, ((uint32_t)h.kind << 24) | ((uint32_t)(hit_id(S, h) + 1) & 0xFFFFFFu));
      if (h.kind != kHitNone) {
        t += h.t * S.ic[region];
        w *= exp_ool(-(S.a[region] * h.t));
        x = o + d * h.t;
        if (h.kind == kHitArray) {
          const double half = 0.5 * (double)P.n_elem * P.pitch;
          if (delta && fabs(x.x) < half && fabs(x.y) < 0.5 * P.elem_h) {
            int e = (int)floor((x.x + half) / P.pitch);
            e = min(max(e, 0), P.n_elem - 1);
            if (kAudit) hsum += event_mix(kEvArray, k, (uint32_t)e);
            const double fd = rx_directivity(P, -d.z);
            Deposit dp;
            if (fd > 0.0) {   // few per launch: added to the histogram directly
              ++n_dep;
              if (make_deposit((uint32_t)((a.tx_base + txl) * P.n_elem + e), P.n_t, P.fs, t, w * fd, &dp))
                add_deposit(a.h, P.n_t, dp, a.hist_scale, a.hist_over);
            }
          } else if (kAudit) {
            hsum += event_mix(kEvArray, k, 0xFFFFFFu);
          }
        } else if (k <= a.max_bounces) {
          ++n_int;
          const Surface sf = surface_of(S, h, x, region);
          const Coef f = coefficients(d, sf.n, S.c[region], S.Z[region], S.c[sf.other], S.Z[sf.other]);
          const Draw v = draw(a.seed, rid, a.tx.id[txl], (uint32_t)k);
          if (sf.kd > 0.0) {
            // receiver-directed secondary ray: weight of everything but the
            // crossings; the march runs in k_secondary
            nee_e = min((int)(v.u3 * (double)P.n_elem), P.n_elem - 1);
            const d3 dv = d3{elem_x(P, nee_e), 0.0, 0.0} - x;
            const double r = sqrt(dot(dv, dv));
            const d3 we = dv * (1.0 / r);
            const double cos_o = dot(f.nr, we);
            if (cos_o <= 0.0) {
              if (kAudit) hsum += event_mix(kEvNee, k, (uint32_t)nee_e | (1u << 16));
            } else {
              const double cos_el = -we.z;
              const double fd = rx_directivity(P, cos_el);
              if (fd == 0.0) {
                if (kAudit) hsum += event_mix(kEvNee, k, (uint32_t)nee_e | (2u << 16));
              } else {
                nee_amp = w * f.Ar * (sf.kd / kPi) * cos_o *
                          (P.elem_w * P.elem_h * cos_el / (r * r)) * (double)P.n_elem * fd;
                push_nee = true;
              }
            }
          }
          // branch on the energy split; weight times coefficient / probability
          const double p_spec = (1.0 - sf.kd) * f.RE;
          uint32_t branch;
          bool alive = true;
          if (v.u0 < p_spec) {
            if (sf.rho > 0.0) {   // glossy about a GGX microfacet; deposits like a mirror path
              const Glossy gl = glossy_reflect(d, f, sf.rho, v.u1, v.u2);
              d = gl.dir;
              w *= f.Ar / f.RE * gl.g;
              alive = gl.ok;
            } else {
              d = d + f.nr * (2.0 * f.ci);
              w *= f.Ar / f.RE;
            }
            delta = true; branch = alive ? 0 : 3;
          } else if (v.u0 < f.RE) {
            // cosine lobe about n_r in the frame of Duff et al. (JCGT 2017)
            const d3 n = f.nr;
            const double sg = n.z >= 0.0 ? 1.0 : -1.0;
            const double aa = -1.0 / (sg + n.z);
            const double bb = n.x * n.y * aa;
            const d3 b1{1.0 + sg * n.x * n.x * aa, sg * bb, -sg * n.x};
            const d3 b2{bb, sg + n.y * n.y * aa, -n.y};
            const double phi = 2.0 * kPi * v.u1, rr = sqrt(v.u2);
            const SinCos sc = sincos_ool(phi);
            const double lx = rr * sc.c, ly = rr * sc.s, lz = sqrt(1.0 - v.u2);
            d = b1 * lx + b2 * ly + n * lz;
            w *= f.Ar / f.RE;
            delta = false; branch = 1;
          } else {
            const double eta = S.c[sf.other] / S.c[region];
            d = d * eta + f.nr * (eta * f.ci - f.ct);
            w *= f.At / (1.0 - f.RE);
            region = sf.other;
            delta = true; branch = 2;
          }
          if (kAudit) hsum += event_mix(kEvBranch, k, branch | (f.tir ? 0x10u : 0u));
          keep = alive;
        }
      }
      if (kAudit && hsum) atomicAdd(a.hash + (long)(a.tx_base + txl) * a.ray_count + (rid - a.ray_begin), (unsigned long long)hsum);
    }

    const Slots sl = block_append2(keep, push_nee, &a.counts[k], scan);
    const long slot = sl.a;
    if (slot >= 0) {
      a.qout.ox[slot] = x.x; a.qout.oy[slot] = x.y; a.qout.oz[slot] = x.z;
      a.qout.dx[slot] = d.x; a.qout.dy[slot] = d.y; a.qout.dz[slot] = d.z;
      a.qout.t[slot] = t; a.qout.w[slot] = w;
      a.qout.rid[slot] = rid;
      a.qout.meta[slot] = (uint32_t)region | ((uint32_t)delta << 8) | ((uint32_t)txl << 12);
    }
    const long ns = sl.b;
    if (ns >= 0) {
      const uint32_t meta = (uint32_t)incident_region | ((uint32_t)nee_e << 8);
      uint32_t key = 0, rank = 0;
      if (a.sort.keys > 0) {   // counted for the sort of the receiver segments
        key = a.sort.key(x.x, x.z, nee_e);
        rank = atomicAdd(a.sort_count + key, 1u);
      }
      a.nee.rec[ns] = SecRec{x.x, x.y, x.z, t, nee_amp, rid, meta, (uint32_t)txl | ((uint32_t)k << 16), key, rank, 0u};
    }
  }
  if (a.counters) flush_counters(a.counters, n_seg, 0, n_dep, n_int, 0);
}

// Receiver-directed secondary rays spawned at interaction k: straight to the
// element centre through every crossed interface (transmission coefficient
// each, zero on total internal reflection), attenuation and travel time per
// medium, then the deposit. The crossings of a segment come from one
// hierarchy walk that keeps the nearest few (receiver_march).
template <bool kAudit, bool kMeshes>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMeshes ? 4 : 5, 8))) void k_secondary(TraceArgs a, int k) {
  const long n_in = (long)(a.counts[k] >> 32);
  if ((long)blockIdx.x * blockDim.x >= n_in) return;   // whole block idle
  __shared__ SceneLDS S;
  extern __shared__ int bvh_stack[];
  load_scene(S, a.scene);
  int* stk = bvh_stack + threadIdx.x;
  const ProbeView& P = a.probe;
  unsigned long long n_seg = 0, n_dep = 0, n_rays = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (long)gridDim.x * blockDim.x) {
    ++n_rays;
    const SecRec q = a.nee.rec[a.sort.keys > 0 ? (long)a.sort_perm[i] : i];
    const d3 x{q.x, q.y, q.z};
    double tof = q.t, amp = q.amp;
    const uint32_t meta = q.meta, txk = q.txk;
    const int reg = meta & 0xFF;
    const int e2 = (int)(meta >> 8);
    const int txl = (int)(txk & 0xFFFF);
    const d3 dv = d3{elem_x(P, e2), 0.0, 0.0} - x;
    const double r = sqrt(dot(dv, dv));
    const d3 we = dv * (1.0 / r);
    const March mr = receiver_march<kMeshes>(S, x, we, r, reg, tof, stk,
                                             [](int, double, int, const Surface&, const Coef&) {});
    n_seg += mr.reached ? mr.crossings + 1 : mr.crossings;   // one segment per leg
    const uint32_t crossings = (uint32_t)mr.crossings;
    const bool blocked = !mr.reached;
    tof = mr.tof;
    amp *= mr.trans;
    Deposit dp;
    bool rec = false;
    if (!blocked) {
      ++n_dep;
      amp *= exp_ool(-mr.att);   // the attenuation of all legs at once
      rec = make_deposit((uint32_t)((a.tx_base + txl) * P.n_elem + e2), P.n_t, P.fs, tof, amp, &dp);
    }
    // record for the binned splat (one atomic per wave on this block's shard
    // of the record buffer), else add directly
    const int shard = blockIdx.x % kDepShards;
    const long shard_cap = a.dep_cap / kDepShards;
    const long slot = wave_append(rec && shard_cap > 0, a.dep_count + shard);
    if (slot >= 0 && slot < shard_cap) {
      const long at = (long)shard * shard_cap + slot;
      a.dep.key[at] = ((dp.row - a.dep.row0) << kDepBinBits) | (uint32_t)(dp.j0 + 1);
      a.dep.w[at] = make_float2(dp.w0, dp.w1);
    } else if (rec) {
      add_deposit(a.h, P.n_t, dp, a.hist_scale, a.hist_over);
    }
    if (kAudit) {
      const uint32_t word = blocked ? ((uint32_t)e2 | (3u << 16) | (crossings << 20))
                                    : ((uint32_t)e2 | (crossings << 20));
      atomicAdd(a.hash + (long)(a.tx_base + txl) * a.ray_count + (q.rid - a.ray_begin),
                (unsigned long long)event_mix(kEvNee, txk >> 16, word));
    }
  }
  if (a.counters) flush_counters(a.counters, 0, n_seg, n_dep, 0, n_rays);
}

// Exclusive scan in place over kSortBlocks contiguous tiles: tile sums, their
// scan (one block), then each tile scanned from its offset.
__device__ __forceinline__ uint32_t block_scan256(uint32_t v, uint32_t* total) {
  __shared__ uint32_t part[256];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele scan
    const uint32_t u = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += u;
    __syncthreads();
  }
  const uint32_t r = part[threadIdx.x] - v;
  *total = part[255];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_sort_tile_sums(const uint32_t* count, int n, uint32_t* part) {
  const int per = (n + kSortBlocks - 1) / kSortBlocks;
  const int b = blockIdx.x * per, e = min(n, b + per);
  uint32_t s = 0;
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) s += count[i];
  uint32_t tot;
  block_scan256(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_sort_tile_offsets(uint32_t* part) {
  uint32_t tot;
  part[threadIdx.x] = block_scan256(part[threadIdx.x], &tot);   // kSortBlocks == 256
}

__global__ __launch_bounds__(256) void k_sort_tile_scan(uint32_t* count, int n, const uint32_t* part) {
  const int per = (n + kSortBlocks - 1) / kSortBlocks;
  const int b = blockIdx.x * per, e = min(n, b + per);
  uint32_t base = part[blockIdx.x];
  for (int i0 = b; i0 < e; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    const uint32_t c = i < e ? count[i] : 0u;
    uint32_t tot;
    const uint32_t x = block_scan256(c, &tot);
    if (i < e) count[i] = base + x;
    base += tot;
  }
}

// Receiver segments of interaction k in key order: index i to its key's
// offset plus its rank (counted by the bounce kernel as it queued the record;
// the order within a key is the atomics' order, and nothing downstream
// depends on it: deposits are integer sums, counters and hashes are sums).
__global__ __launch_bounds__(256) void k_sec_scatter(TraceArgs a, int k) {
  const long n_in = (long)(a.counts[k] >> 32);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += (long)gridDim.x * blockDim.x) {
    const uint2 kr = *reinterpret_cast<const uint2*>(&a.nee.rec[i].key);
    a.sort_perm[a.sort_count[kr.x] + kr.y] = (uint32_t)i;
  }
}

// rf[row][k] = sum_{|m| <= M} h[row][k - m] s[m]  (Eq. axial_sig as a FIR on
// the deposit histogram; h is zero outside [0, n_t)). One block computes a
// tile of kPulseTile outputs of one row from an LDS copy of the tile + halo
// (fir_block: kPulseR outputs per thread).
constexpr int kPulseTile = 256 * kPulseR;

// Samples of the FIR's input: an fp32 row, or the fixed-point histogram
// read out (units times 1 / scale, a power of two; NaN once a weight was clamped).
struct PulseIn {
  const float* f;
  const long long* q;
  double inv_scale;
  const unsigned long long* over;
  __device__ __forceinline__ float at(long i, bool bad) const {
    if (f) return f[i];
    return bad ? __builtin_nanf("") : (float)((double)q[i] * inv_scale);
  }
};

template <bool kVec>
__global__ __launch_bounds__(256) void k_pulse(PulseIn in, float* __restrict__ rf,
                                               const float* __restrict__ taps, int M, int n_t,
                                               int tiles_per_row) {
  // x[i] = h[k0 - M + i]; c[q] = s[M - q] = taps[2M - q], zero-padded to Tp
  __shared__ __align__(16) float x[kPulseTile + 2 * kMaxTaps];
  __shared__ __align__(16) float c[2 * kMaxTaps];
  const long row = blockIdx.x / tiles_per_row;
  const int k0 = (blockIdx.x % tiles_per_row) * kPulseTile;
  const long r0 = row * (long)n_t;
  const bool bad = in.over && *in.over != 0ull;
  const int T = 2 * M + 1, Tp = fir_padded(M);
  for (int j = threadIdx.x; j < kPulseTile + Tp; j += blockDim.x) {
    const int src = k0 - M + j;
    x[j] = (src >= 0 && src < n_t) ? in.at(r0 + src, bad) : 0.0f;
  }
  for (int j = threadIdx.x; j < Tp; j += blockDim.x) c[j] = j < T ? taps[2 * M - j] : 0.0f;
  __syncthreads();
  // output k0 + b + r = sum_q x[b + r + q] c[q]
  const int b = threadIdx.x * kPulseR;
  float acc[kPulseR];
  fir_block(x, c, b, Tp, acc);
  fir_store<kVec>(rf + row * (long)n_t, k0 + b, n_t, acc);
}

__global__ void k_fill_u32(uint32_t* p, long n, uint32_t v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- launchers
static int grid_for(long n, int per_block, int cap) {
  long g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

void launch_fill_u32(uint32_t* p, long n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
}

// Grids are capped at a few blocks per compute unit; the kernels loop.
constexpr int kMaxBlocks = 8192;

static size_t stack_bytes(const TraceArgs& a) {
  return a.scene.n_meshes > 0 ? (size_t)a.scene.stack_cap * 256 * sizeof(int) : 0;
}

void launch_bounce(const TraceArgs& a, int k, long max_rays, bool audit, hipStream_t s) {
  const dim3 grid(grid_for(max_rays, 256, kMaxBlocks)), block(256);
  const bool m = a.scene.n_meshes > 0;
  const auto kern = audit ? (m ? k_bounce<true, true> : k_bounce<true, false>)
                          : (m ? k_bounce<false, true> : k_bounce<false, false>);
  hipLaunchKernelGGL(kern, grid, block, stack_bytes(a), s, a, k);
}

void launch_secondary(const TraceArgs& a, int k, long max_rays, bool audit, hipStream_t s) {
  const dim3 grid(grid_for(max_rays, 256, kMaxBlocks)), block(256);
  const bool m = a.scene.n_meshes > 0;
  const auto kern = audit ? (m ? k_secondary<true, true> : k_secondary<true, false>)
                          : (m ? k_secondary<false, true> : k_secondary<false, false>);
  hipLaunchKernelGGL(kern, grid, block, stack_bytes(a), s, a, k);
}

void launch_sort_offsets(uint32_t* count, int n, uint32_t* part, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_tile_sums, dim3(kSortBlocks), dim3(256), 0, s, count, n, part);
  hipLaunchKernelGGL(k_sort_tile_offsets, dim3(1), dim3(kSortBlocks), 0, s, part);
  hipLaunchKernelGGL(k_sort_tile_scan, dim3(kSortBlocks), dim3(256), 0, s, count, n, part);
}

void launch_secondary_sort(const TraceArgs& a, int k, long max_rays, hipStream_t s) {
  if (a.sort.keys <= 0) return;
  launch_sort_offsets(a.sort_count, a.sort.keys, a.sort_part, s);
  hipLaunchKernelGGL(k_sec_scatter, dim3(grid_for(max_rays, 256, kMaxBlocks)), dim3(256), 0, s, a, k);
}

static int pulse(const PulseIn& in, float* rf, const float* taps, int M, int n_t, long n_rows, hipStream_t s) {
  if (M > kMaxTaps - 1) return -1;
  const int tiles = (n_t + kPulseTile - 1) / kPulseTile;
  // 16-byte stores when every row starts 16-byte aligned
  const bool vec = n_t % 4 == 0 && ((uintptr_t)rf & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(k_pulse<true>, dim3((unsigned)(n_rows * tiles)), dim3(256), 0, s, in, rf, taps, M, n_t,
                       tiles);
  else
    hipLaunchKernelGGL(k_pulse<false>, dim3((unsigned)(n_rows * tiles)), dim3(256), 0, s, in, rf, taps, M, n_t,
                       tiles);
  return 0;
}

int launch_pulse(const float* h, float* rf, const float* taps, int M, int n_t, long n_rows, hipStream_t s) {
  return pulse(PulseIn{h, nullptr, 0.0, nullptr}, rf, taps, M, n_t, n_rows, s);
}

int launch_pulse_fixed(const long long* h, double hist_scale, const unsigned long long* hist_over, float* rf,
                       const float* taps, int M, int n_t, long n_rows, hipStream_t s) {
  return pulse(PulseIn{nullptr, h, 1.0 / hist_scale, hist_over}, rf, taps, M, n_t, n_rows, s);
}

}  // namespace usrt
