// Backward of the transport by path replay (paper Sec. 3.2, Eq. chain_rule):
// for fixed random numbers, every ray's path is traced again from its Philox
// counters with exactly the forward's decisions, and the gradient of
//   L = sum over deposits of <dL/dh, tent(t fs) a>
// with respect to the scene parameters is accumulated by reverse-mode
// differentiation along the path. Nothing is stored between the forward and
// the backward call. Inside this call the rays of a chunk are traced again as
// a wavefront (one launch per step, survivors compacted), each step leaving
// the exact fp64 state before it in an 80-byte record of its ray; the
// secondary rays of the diffuse interactions are differentiated next, and
// one thread per ray finally sweeps its records backwards. Discrete choices
// (branch, hit surface, element, total internal reflection, sample index)
// are frozen; branch probabilities are sampling densities and carry no
// derivative.
//
// Every adjoint sum (parameters, mesh vertices, acquisition parameters) is
// kept in the order-independent integer windows of sum_add: per block in LDS,
// then added into one global accumulator per entry, read out once per call.
// Identical calls therefore give bitwise identical gradients whatever the
// scheduling of the threads and their atomics.
#include "geometry.h"
#include "kernels.h"

namespace usrt {

namespace {

// Per-block sums of the region, plane, sphere, cylinder and roughness
// adjoints (the first n_grad entries of theta; mesh coefficients go through
// the per-vertex sums) live in LDS as grad_copies interleaved copies of
// n_grad accumulators of kSumWords words: a lane adds to copy
// lane % grad_copies, so lanes adding to the same parameter contend at most
// 64 / grad_copies ways. The copies are added up word by word when the
// block ends and the totals go into the global accumulators with integer
// atomics (order-independent).
__device__ __forceinline__ int grad_words(int n_grad) { return n_grad * kSumWords; }

__device__ __forceinline__ void words_clear(unsigned long long* w, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) w[j] = 0ull;
}

__device__ __forceinline__ void grad_flush(const unsigned long long* gsh, int n_grad, int copies,
                                           unsigned long long* g_sum) {
  const int n = grad_words(n_grad);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    unsigned long long v = 0ull;
    for (int c = 0; c < copies; ++c) v += gsh[c * n + j];
    if (v) atomicAdd(g_sum + j, v);
  }
}

// Mesh vertex sums staged in LDS: an open-addressing table per block, keyed
// by (vertex, window of the value's leading bit), each entry holding the
// two words a value adds to (window b and b - 1). The lanes of a block that
// add to the same vertex at about the same time meet in one entry, and vh_flush adds the entries to the block's global copy at
// points where the block is synchronised. The words are integers, so the
// totals are those of adding every value straight to the global copy.
// The table has 2^bits entries: 2^11 in the reverse sweep, 2^9 in the
// secondary phase, whose crossing caches and stacks leave less LDS.
constexpr int kVhBitsReverse = 11, kVhBitsSecondary = 9;
constexpr uint32_t kVhEmpty = 0xFFFFFFFFu;   // vertex indices stay below 2^28
constexpr int kVhProbes = 8;                 // entries tried before going to the global copy
constexpr size_t vh_bytes(int bits) {
  return ((size_t)1 << bits) * (sizeof(uint32_t) + 2 * sizeof(unsigned long long));
}
// Empties the table (keys [n], then words [2][n]); the caller synchronises.
__device__ __forceinline__ void vh_clear(uint32_t* hk, unsigned long long* hw, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    hk[j] = kVhEmpty;
    hw[j] = 0ull;
    hw[n + j] = 0ull;
  }
}
// Called by every thread of the block: the table's entries added to the
// block's vertex sums in HBM and the table emptied.
__device__ __forceinline__ void vh_flush(uint32_t* hk, unsigned long long* hw, unsigned long long* vadj, long vstride,
                                         int n) {
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t key = hk[j];
    if (key != kVhEmpty) {
      const long v = key >> 4;
      const int b = key & 15;
      const unsigned long long w0 = hw[j], w1 = hw[n + j];
      if (w0) atomicAdd(vadj + b * vstride + v, w0);
      if (w1) atomicAdd(vadj + (b - 1) * vstride + v, w1);
      hk[j] = kVhEmpty;
      hw[j] = 0ull;
      hw[n + j] = 0ull;
    }
  }
  __syncthreads();
}
// Per-block gradient accumulator over the flat parameter vector.
struct GradAcc {
  unsigned long long* g;          // this lane's LDS copy: [n_grad][kSumWords]
  int n_regions, n_planes, n_spheres, n_cylinders;
  double np_per_m;
  const double* vnormal;
  unsigned long long* vadj;       // this block's copy of the vertex sums (HBM): [kSumWords][vstride]
  long vstride;
  uint32_t* hk = nullptr;         // optional LDS table of vertex sums (2^vh_bits keys, then twice as many words)
  unsigned long long* hw = nullptr;
  int vh_bits = 0;
  __device__ void add(int j, double v) { sum_add(g + (long)j * kSumWords, v); }
  // adjoint vbar of mesh vertex v: v = v_rest + (sum_j q_j phi_j(v)) n(v), so
  // the vertex contributes (vbar . n(v)) phi_j(v) to q_j; the scalar is summed
  // per vertex here and projected onto the basis once per call
  __device__ void mesh_vertex(int v, int m, d3 vbar) {
    (void)m;
    const double s = vbar.x * vnormal[3 * v] + vbar.y * vnormal[3 * v + 1] + vbar.z * vnormal[3 * v + 2];
    if (!hk) {
      sum_add(vadj + v, vstride, s);
      return;
    }
    // the value's two words into its table entry (linear probing), or
    // straight to the global copy when the entries tried are taken
    SumPieces p;
    if (!sum_pieces(s, &p)) return;
    if (p.over) {
      atomicAdd(vadj + kSumBins * vstride + v, 1ull);
      return;
    }
    const uint32_t key = ((uint32_t)v << 4) | (uint32_t)p.b;
    const uint32_t vh_n = 1u << vh_bits;
    uint32_t slot = (key * 2654435761u) >> (32 - vh_bits);
    for (int t = 0; t < kVhProbes; ++t) {
      const uint32_t prev = atomicCAS(hk + slot, kVhEmpty, key);
      if (prev == kVhEmpty || prev == key) {
        atomicAdd(hw + slot, p.hi);
        if (p.lo) atomicAdd(hw + vh_n + slot, p.lo);
        return;
      }
      slot = (slot + 1) & (vh_n - 1);
    }
    atomicAdd(vadj + p.b * vstride + v, p.hi);   // the table is crowded here
    if (p.lo) atomicAdd(vadj + (p.b - 1) * vstride + v, p.lo);
  }
  __device__ void c(int r, double v) { add(3 * r, v); }
  __device__ void Z(int r, double v) { add(3 * r + 1, v); }
  // v is the adjoint of the amplitude attenuation a [Np/m]; a = alpha * np_per_m
  __device__ void a(int r, double v) { add(3 * r + 2, v * np_per_m); }
  __device__ void plane(int k, double v) { add(3 * n_regions + k, v); }
  // roughness of plane / sphere / cylinder k or of mesh k (hit kind decides)
  __device__ void rough(int kind, int k, double v) {
    const int base = 3 * n_regions + n_planes + 4 * n_spheres + 3 * n_cylinders;
    const int j = kind == kHitPlane ? k
                : kind == kHitSphere ? n_planes + k
                : kind == kHitCylinder ? n_planes + n_spheres + k
                : n_planes + n_spheres + n_cylinders + k;
    add(base + j, v);
  }
  __device__ void cylinder(int k, double xbar, double zbar, double rbar) {
    const int j = 3 * n_regions + n_planes + 4 * n_spheres + 3 * k;
    add(j, xbar);
    add(j + 1, zbar);
    add(j + 2, rbar);
  }
  __device__ void sphere(int k, d3 cbar, double rbar) {
    const int j = 3 * n_regions + n_planes + 4 * k;
    add(j, cbar.x);
    add(j + 1, cbar.y);
    add(j + 2, cbar.z);
    add(j + 3, rbar);
  }
};

__device__ __forceinline__ d3 operator-(d3 a) { return {-a.x, -a.y, -a.z}; }

// Adjoints of one crossing's triangle collected from its distance and its
// normal, so that the three vertices take one atomic update each.
struct TriAdj {
  d3 nub{0, 0, 0};    // adjoint of nu = (p1 - p0) x (p2 - p0)
  d3 p0b{0, 0, 0};    // direct adjoint of p0
};

// Adjoint through nu = (p1 - p0) x (p2 - p0) into the three vertices.
__device__ __forceinline__ void tri_nu_backward(const SceneLDS& S, int i, d3 nub, d3 p0b_extra,
                                                GradAcc& G) {
  const int4 tv = gload(S.tri + i);
  const d3 p0 = vtx(S.vcur, tv.x), e1 = vtx(S.vcur, tv.y) - p0, e2 = vtx(S.vcur, tv.z) - p0;
  const d3 e1b = cross(e2, nub), e2b = cross(nub, e1);
  G.mesh_vertex(tv.x, tv.w, p0b_extra - e1b - e2b);
  G.mesh_vertex(tv.y, tv.w, e1b);
  G.mesh_vertex(tv.z, tv.w, e2b);
}

// Adjoint of G1(c, rho) (Smith masking for GGX): adds gbar dG1/dc to *cbar
// and gbar dG1/drho to *rhobar.
__device__ __forceinline__ void smith_g1_vjp(double c, double rho, double gbar, double* cbar, double* rhobar) {
  const double s = sqrt(rho * rho + (1.0 - rho * rho) * c * c);
  const double den = c + s;
  const double inv2 = 1.0 / (den * den);
  *cbar += gbar * 2.0 * (s - c * (1.0 - rho * rho) * c / s) * inv2;
  *rhobar += gbar * (-2.0 * c * (rho * (1.0 - c * c) / s)) * inv2;
}

// d/dc of the receive directivity (Eq. cutoff) at cosine c; zero outside the ramp.
__device__ __forceinline__ double rx_directivity_deriv(const ProbeView& p, double cos_a) {
  const double c = fmin(1.0, fmax(-1.0, cos_a));
  const double al = acos_ool(c);
  if (al <= p.alpha_m || al > p.alpha_c) return 0.0;
  const double s = sqrt(fmax(0.0, 1.0 - c * c));
  return s > 0.0 ? 1.0 / ((p.alpha_c - p.alpha_m) * s) : 0.0;
}

// Adjoints (g_a, g_t) of a deposit (t, a) given dL/dh on its row: the tent
// deposits a (1 - f) at j0 = floor(t fs) and a f at j0 + 1.
__device__ __forceinline__ void tent_adjoint(const float* row, int n_t, double fs, double t,
                                             double a, double* ga, double* gt) {
  const double x = t * fs;
  if (!(x > -1.0 && x < (double)n_t)) { *ga = 0.0; *gt = 0.0; return; }
  const double j0d = floor(x);
  const double f = x - j0d;
  const int j0 = (int)j0d;
  const double g0 = j0 >= 0 ? (double)row[j0] : 0.0;
  const double g1 = j0 + 1 < n_t ? (double)row[j0 + 1] : 0.0;
  *ga = g0 * (1.0 - f) + g1 * f;
  *gt = a * fs * (g1 - g0);
}

// Adjoint of a distance s along (o, d) to the surface of `h`, for a plane
// s = (z_p - o.z) / d.z, the array face s = -o.z / d.z, or a sphere
// s = -b + sig sqrt(b^2 - cc), b = (o - C).d, cc = |o - C|^2 - R^2.
__device__ __forceinline__ void distance_backward(const SceneLDS& S, int kind, int idx, double sig,
                                                  d3 o, d3 d, double s, double sbar, d3& obar,
                                                  d3& dbar, GradAcc& G, TriAdj& ta) {
  if (sbar == 0.0) return;
  if (kind == kHitMesh) {   // s = nu.(p0 - o) / nu.d
    const int4 tv = gload(S.tri + idx);
    const d3 p0 = vtx(S.vcur, tv.x);
    const d3 nu = cross(vtx(S.vcur, tv.y) - p0, vtx(S.vcur, tv.z) - p0);
    const double den = dot(nu, d);
    const double numb = sbar / den, denb = -sbar * s / den;
    obar = obar - nu * numb;
    dbar = dbar + nu * denb;
    ta.nub = ta.nub + (p0 - o) * numb + d * denb;
    ta.p0b = ta.p0b + nu * numb;
    return;
  }
  if (kind == kHitPlane || kind == kHitArray) {
    const double inv = 1.0 / d.z;
    if (kind == kHitPlane) G.plane(idx, sbar * inv);
    obar.z -= sbar * inv;
    dbar.z -= sbar * s * inv;
  } else if (kind == kHitCylinder) {
    // s = (-b + sig q) / a, q = sqrt(b^2 - a cc), a = dx^2 + dz^2,
    // b = ox dx + oz dz, cc = ox^2 + oz^2 - R^2 in the x-z plane
    const double ox = o.x - S.cx[idx], oz = o.z - S.cz[idx];
    const double a = d.x * d.x + d.z * d.z;
    const double b = ox * d.x + oz * d.z;
    const double cc = ox * ox + oz * oz - S.cr[idx] * S.cr[idx];
    const double q = sqrt(fmax(b * b - a * cc, 0.0));
    if (q == 0.0) return;   // tangent ray: measure zero
    const double bbar = sbar * (-1.0 + sig * b / q) / a;
    const double ccbar = sbar * (-sig / (2.0 * q));
    const double abar = -sbar * (sig * cc / (2.0 * q) + s) / a;
    const double oxbar = bbar * d.x + 2.0 * ccbar * ox, ozbar = bbar * d.z + 2.0 * ccbar * oz;
    dbar.x += bbar * ox + 2.0 * abar * d.x;
    dbar.z += bbar * oz + 2.0 * abar * d.z;
    obar.x += oxbar;
    obar.z += ozbar;
    G.cylinder(idx, -oxbar, -ozbar, -2.0 * ccbar * S.cr[idx]);
  } else {
    const d3 oc{o.x - S.sx[idx], o.y - S.sy[idx], o.z - S.sz[idx]};
    const double b = dot(oc, d);
    const double cc = dot(oc, oc) - S.sr[idx] * S.sr[idx];
    const double q = sqrt(fmax(b * b - cc, 0.0));
    if (q == 0.0) return;   // tangent ray: measure zero
    const double bbar = sbar * (-1.0 + sig * b / q);
    const double ccbar = sbar * (-sig / (2.0 * q));
    const d3 ocbar = d * bbar + oc * (2.0 * ccbar);
    dbar = dbar + oc * bbar;
    obar = obar + ocbar;
    G.sphere(idx, -ocbar, -2.0 * ccbar * S.sr[idx]);
  }
}

// Root sign of the primary intersection with cylinder idx, as the forward chose it.
__device__ __forceinline__ double cylinder_root(const SceneLDS& S, int idx, d3 o, d3 d) {
  const double ox = o.x - S.cx[idx], oz = o.z - S.cz[idx];
  const double a = d.x * d.x + d.z * d.z;
  const double b = ox * d.x + oz * d.z;
  const double disc = b * b - a * (ox * ox + oz * oz - S.cr[idx] * S.cr[idx]);
  return ((-b - sqrt(disc)) / a > kTMin) ? -1.0 : 1.0;
}

// Root sign of the primary intersection, as the forward chose it.
__device__ __forceinline__ double primary_root(const SceneLDS& S, int idx, d3 o, d3 d) {
  const d3 oc{o.x - S.sx[idx], o.y - S.sy[idx], o.z - S.sz[idx]};
  const double b = dot(oc, d);
  const double disc = b * b - (dot(oc, oc) - S.sr[idx] * S.sr[idx]);
  const double q = sqrt(disc);
  return (-b - q > kTMin) ? -1.0 : 1.0;
}

// Adjoint of the geometric normal at x on the hit surface (plane: constant;
// sphere: n = (x - C) / R). nbar is the adjoint of n; adds to xbar.
__device__ __forceinline__ void normal_backward(const SceneLDS& S, int kind, int idx, d3 n,
                                                d3 nbar, d3& xbar, GradAcc& G, TriAdj& ta) {
  if (kind == kHitMesh) {   // n = nu / |nu|
    const int4 tv = gload(S.tri + idx);
    const d3 p0 = vtx(S.vcur, tv.x);
    const d3 nu = cross(vtx(S.vcur, tv.y) - p0, vtx(S.vcur, tv.z) - p0);
    ta.nub = ta.nub + (nbar - n * dot(nbar, n)) * (1.0 / sqrt(dot(nu, nu)));
    return;
  }
  if (kind == kHitCylinder) {   // n = ((x - cx) / R, 0, (z - cz) / R)
    const double ir = 1.0 / S.cr[idx];
    const double tx = nbar.x * ir, tz = nbar.z * ir;
    xbar.x += tx;
    xbar.z += tz;
    G.cylinder(idx, -tx, -tz, -(nbar.x * n.x + nbar.z * n.z) * ir);
    return;
  }
  if (kind != kHitSphere) return;
  const double ir = 1.0 / S.sr[idx];
  const d3 t = nbar * ir;
  xbar = xbar + t;
  G.sphere(idx, -t, -dot(nbar, n) * ir);
}

// Adjoint of the pressure coefficients and of cos theta_t: given Abar (total
// adjoint on A_r and A_t, which differ by the constant 1), ctbar and etabar,
// returns cibar and adds the impedance and sound-speed adjoints.
__device__ __forceinline__ double interface_backward(const Coef& f, double eta, int r1, int r2,
                                                     double Z1, double Z2, double c1, double Abar,
                                                     double ctbar, double etabar, GradAcc& G) {
  double cibar = 0.0;
  if (!f.tir) {
    const double u = Z2 * f.ci, v = Z1 * f.ct, D = u + v;
    const double ubar = Abar * 2.0 * v / (D * D);
    const double vbar = -Abar * 2.0 * u / (D * D);
    G.Z(r2, ubar * f.ci);
    cibar += ubar * Z2;
    G.Z(r1, vbar * f.ct);
    ctbar += vbar * Z1;
    if (f.ct > 0.0 && ctbar != 0.0) {   // ct = sqrt(1 - eta^2 (1 - ci^2))
      const double s2bar = -ctbar / (2.0 * f.ct);
      etabar += s2bar * 2.0 * eta * (1.0 - f.ci * f.ci);
      cibar += s2bar * (-2.0 * eta * eta * f.ci);
    }
  }
  if (etabar != 0.0) {   // eta = c2 / c1
    G.c(r2, etabar / c1);
    G.c(r1, -etabar * eta / c1);
  }
  return cibar;
}

// Crossings of a receiver segment remembered between the two passes of its
// adjoint (their distance from the segment's start and hit word, in LDS,
// interleaved across the block's threads); further crossings are found again.
constexpr int kLegCache = kMarchLegs;

struct ReplayCtx {
  const SceneLDS& S;
  const ProbeView& P;
  const float* gh;      // dL/dh rows [n_tx][n_elem][n_t]
  const float* ghf;     // the same for the pulse's derivative in f0, or null
  long row_base;        // (tx_base + txl) * n_elem
  GradAcc& G;
  int* stk;             // this thread's hierarchy stack in LDS
  double* leg_t;        // this thread's crossing cache in LDS: distance from x ...
  int* leg_h;           // ... and kind << 28 | index
  MarchRecs rec;        // the marches a recorded forward made ...
  long rq;              // ... this one's entry, or -1 (march again)
};

// Secondary ray of interaction k at x (weight watt, time tp, interface f):
// adds its adjoints to xbar, nrbar, Arbar, wattbar, tpbar, the target
// element's x (xebar), f0 through the pulse (f0bar) and the parameters.
template <bool kMeshes>
__device__ void secondary_backward(ReplayCtx& C, int region, d3 x, const Coef& f, double kd,
                                   double watt, double tp, int e2, d3& xbar, d3& nrbar,
                                   double& Arbar, double& wattbar, double& tpbar, double& xebar,
                                   double& f0bar) {
  const SceneLDS& S = C.S;
  const ProbeView& P = C.P;
  const double xe = ((double)e2 - 0.5 * (double)(P.n_elem - 1)) * P.pitch;
  const d3 dv = d3{xe, 0.0, 0.0} - x;
  const double r = sqrt(dot(dv, dv));
  const d3 we = dv * (1.0 / r);
  const double co = dot(f.nr, we);
  if (co <= 0.0) return;
  const double cel = -we.z;
  const double fd = rx_directivity(P, cel);
  if (fd == 0.0) return;
  const double K = (kd / kPi) * P.elem_w * P.elem_h * (double)P.n_elem;
  const double amp0 = watt * f.Ar * (kd / kPi) * co * (P.elem_w * P.elem_h * cel / (r * r)) *
                      (double)P.n_elem * fd;
  // pass 1: the march as the forward did it, its crossings cached in LDS
  // (a recorded frame reads the march the forward made instead)
  const int step = blockDim.x;
  March mr;
  if (C.rq >= 0) {
    const MarchRecs& R = C.rec;
    const long q = C.rq;
    const uint32_t ns = R.nstate[q];
    mr = March{R.tof[q], R.att[q], R.trans[q], (int)(ns >> 2), (ns & 3u) == 2u};
    for (int j = 0; j < kLegCache && j < mr.crossings; ++j) {
      C.leg_t[j * step] = R.s[j * R.cap + q];
      C.leg_h[j * step] = R.h[j * R.cap + q];
    }
  } else {
    mr = receiver_march<kMeshes>(
        S, x, we, r, region, tp, C.stk, [&](int j, double sj, int hw, const Surface&, const Coef&) {
          if (j < kLegCache) {
            C.leg_t[j * step] = sj;
            C.leg_h[j * step] = hw;
          }
        });
  }
  if (!mr.reached) return;   // blocked: the forward dropped this deposit
  const int n_cross = mr.crossings;
  const double tof = mr.tof;
  const double rest = mr.trans * exp_ool(-mr.att);   // the attenuation of all legs at once, as the forward
  const double amp = amp0 * rest;
  double GA, GT;
  tent_adjoint(C.gh + (C.row_base + e2) * (long)P.n_t, P.n_t, P.fs, tof, amp, &GA, &GT);
  if (C.ghf) {
    double gf, unused;
    tent_adjoint(C.ghf + (C.row_base + e2) * (long)P.n_t, P.n_t, P.fs, tof, 0.0, &gf, &unused);
    f0bar += gf * amp;
  }
  if (GA == 0.0 && GT == 0.0) return;
  tpbar += GT;
  const double AA = GA * amp;   // adjoint of log(amplitude)
  // pass 2: every leg and crossing, with s_j the distance from x
  d3 webar{0, 0, 0}, xb{0, 0, 0};
  double rbar = 0.0;
  {
    int reg = region;
    double s_prev = 0.0;
    for (int leg = 0;; ++leg) {
      if (leg == n_cross) {   // the final stretch to the element
        const double ell = r - s_prev;
        C.G.c(reg, -GT * ell / (S.c[reg] * S.c[reg]));
        C.G.a(reg, -AA * ell);
        rbar += GT / S.c[reg] - AA * S.a[reg];
        break;
      }
      // crossing `leg`: cached by pass 1, or the nearest beyond the previous one
      double sj;
      int hw;
      if (leg < kLegCache) {
        sj = C.leg_t[leg * step];
        hw = C.leg_h[leg * step];
      } else {
        const SegHits L = segment_hits<kMeshes>(S, x, we, s_prev, r, C.stk);
        sj = L.s[0];
        hw = L.h[0];
      }
      const Hit h{hw >> 28, hw & 0x0FFFFFFF, sj};
      const double ell = sj - s_prev;
      C.G.c(reg, -GT * ell / (S.c[reg] * S.c[reg]));
      C.G.a(reg, -AA * ell);
      s_prev = sj;
      const d3 p = x + we * sj;
      const Surface sf = surface_of(S, h, p, reg);
      const int other = sf.other;
      const Coef g = coefficients(we, sf.n, S.c[reg], S.Z[reg], S.c[other], S.Z[other]);
      const double eta = S.c[other] / S.c[reg];
      // distance s_j: the time and attenuation switch medium there
      double sbar = GT * (1.0 / S.c[reg] - 1.0 / S.c[other]) + AA * (S.a[other] - S.a[reg]);
      // transmission coefficient of the crossing: d log(amp) / d At = 1 / At
      const double cibar = interface_backward(g, eta, reg, other, S.Z[reg], S.Z[other], S.c[reg],
                                              AA / g.At, 0.0, 0.0, C.G);
      // ci = -nr . we
      const d3 nrb = we * (-cibar);
      webar = webar - g.nr * cibar;
      const double sgn = dot(sf.n, we) > 0.0 ? -1.0 : 1.0;
      d3 pbar{0, 0, 0};
      TriAdj ta;
      normal_backward(S, h.kind, h.index, sf.n, nrb * sgn, pbar, C.G, ta);
      // p_j = x + we s_j
      xb = xb + pbar;
      webar = webar + pbar * sj;
      sbar += dot(pbar, we);
      // s_j as a function of (x, we): entering a sphere takes the near root
      double sig = -1.0;
      if (h.kind == kHitSphere) sig = (reg == S.sreg[h.index][1]) ? -1.0 : 1.0;
      if (h.kind == kHitCylinder) sig = (reg == S.creg[h.index][1]) ? -1.0 : 1.0;
      distance_backward(S, h.kind, h.index, sig, x, we, sj, sbar, xb, webar, C.G, ta);
      if (h.kind == kHitMesh) tri_nu_backward(S, h.index, ta.nub, ta.p0b, C.G);
      reg = other;
    }
  }
  // amp0 = watt * Ar * (kd/pi) * co * (A_el cel / r^2) * N_e * fd
  const double A0bar = GA * rest;
  const double base = K * co * cel * fd / (r * r);
  wattbar += A0bar * f.Ar * base;
  Arbar += A0bar * watt * base;
  const double common = A0bar * watt * f.Ar * K / (r * r);
  const double cobar = common * cel * fd;
  const double celbar = common * co * (fd + cel * rx_directivity_deriv(P, cel));
  rbar += A0bar * watt * f.Ar * base * (-2.0 / r);
  nrbar = nrbar + we * cobar;
  webar = webar + f.nr * cobar;
  webar.z -= celbar;
  // we = dv / r, r = |dv|, dv = y - x
  const d3 dvbar = (webar - we * dot(webar, we)) * (1.0 / r) + we * rbar;
  xbar = xbar + xb - dvbar;
  xebar += dvbar.x;   // the element centre y = (x_e, 0, 0) enters as dv = y - x
}

// Ray of chunk slot i: transmit (local index) and ray id.
__device__ __forceinline__ void ray_of(const ReplayArgs& a, long i, int* txl, uint32_t* rid) {
  const long g = a.g0 + i;
  *txl = (int)(g / a.ray_count);
  *rid = (uint32_t)(a.ray_begin + g % a.ray_count);
}

// State after the interaction at x, given the draw v (same decisions as the
// forward); returns false when the path ends.
struct Step {
  Hit h;
  Surface sf;
  Coef f;
  double L, E, tp, watt;
  d3 x;
};

__device__ __forceinline__ Step step_at(const SceneLDS& S, d3 o, d3 d, double t, double w, int region,
                                        const Hit& h) {
  Step st;
  st.h = h;
  st.L = h.t;
  st.E = exp_ool(-(S.a[region] * h.t));
  st.tp = t + h.t * S.ic[region];   // as the forward transport forms it
  st.watt = w * st.E;
  st.x = o + d * h.t;
  if (h.kind != kHitArray && h.kind != kHitNone) {
    st.sf = surface_of(S, h, st.x, region);
    st.f = coefficients(d, st.sf.n, S.c[region], S.Z[region], S.c[st.sf.other], S.Z[st.sf.other]);
  }
  return st;
}

}  // namespace

// Phase 1, one launch per step k as in the forward transport: the live rays
// of the chunk (all of them at k = 1, emitted here) take their step k again,
// keeping the state before it and the surface it hits in the step record of
// their chunk index; the survivors are compacted into the next queue and
// every interaction on a diffuse surface is queued for phase 2.
template <bool kMeshes, bool kDeposit>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_replay_forward(ReplayArgs a, int k, long n) {
  const long n_in = k == 1 ? n : (long)(uint32_t)a.counts[k - 1];   // survivors of step k - 1
  if ((long)blockIdx.x * blockDim.x >= n_in) return;   // whole block idle
  __shared__ SceneLDS S;
  __shared__ unsigned long long scan[8];
  extern __shared__ int bvh_stack[];
  load_scene(S, a.scene);
  int* stk = bvh_stack + threadIdx.x;
  const ProbeView& P = a.probe;
  const int B = a.max_bounces;
  const long cap = a.cap;
  const long stride = (long)gridDim.x * blockDim.x;
  uint32_t n_seg = 0, n_dep = 0, n_int = 0;   // event counters of a recorded forward
  // block-uniform loop: the queue append below synchronises the block
  for (long base = (long)blockIdx.x * blockDim.x; base < n_in; base += stride) {
    const long iq = base + threadIdx.x;
    const bool active = iq < n_in;
    d3 o{0, 0, 0}, d{0, 0, 1};
    double t = 0.0, w = 0.0;
    uint32_t ci = 0;   // chunk index of the ray
    int region = 0;
    bool delta = true, keep = false, diffuse = false;
    uint32_t skey = 0;   // sort key of a diffuse interaction's receiver segment
    if (active) {
      if (k == 1) {
        ci = (uint32_t)iq;
        int txl;
        uint32_t rid;
        ray_of(a, ci, &txl, &rid);
        const int e = (int)(rid / (uint32_t)a.rays_per_elem);
        const Draw u = draw(a.seed, rid, a.tx.id[txl], 0);
        const double sa = a.tx.sin_a[txl], ca = a.tx.cos_a[txl];
        o = d3{((double)e - 0.5 * (double)(P.n_elem - 1)) * P.pitch + (u.u0 - 0.5) * P.elem_w,
               (u.u1 - 0.5) * P.elem_h, 0.0};
        d = d3{sa, 0.0, ca};
        t = o.x * (sa / P.c_ref);
        w = fmax(0.0, ca) / (double)a.rays_per_elem;
        region = S.start_region;
        a.stk.last[ci] = 0;
      } else {
        o = d3{a.qin.ox[iq], a.qin.oy[iq], a.qin.oz[iq]};
        d = d3{a.qin.dx[iq], a.qin.dy[iq], a.qin.dz[iq]};
        t = a.qin.t[iq];
        w = a.qin.w[iq];
        ci = a.qin.rid[iq];
        const uint32_t m = a.qin.meta[iq];
        region = m & 0xFF;
        delta = (m >> 8) & 1u;
      }
      const long at = (long)(k - 1) * cap + ci;
      const Hit h = closest_hit<kMeshes>(S, o, d, true, stk);
      if (kDeposit) ++n_seg;
      a.stk.rec[at] = StepRec{o.x, o.y, o.z, d.x, d.y, d.z, t, w, h.t,
                              (uint32_t)region | ((uint32_t)delta << 8) | ((uint32_t)h.kind << 12),
                              h.index};
      if (h.kind == kHitArray) {
        a.stk.last[ci] = k;
        if (kDeposit) {   // a recorded forward: the array hit's deposit, as the bounce kernel makes it
          const double th = t + h.t * S.ic[region];
          const double wh = w * exp_ool(-(S.a[region] * h.t));
          const d3 x = o + d * h.t;
          const double half = 0.5 * (double)P.n_elem * P.pitch;
          if (delta && fabs(x.x) < half && fabs(x.y) < 0.5 * P.elem_h) {
            int e = (int)floor((x.x + half) / P.pitch);
            e = min(max(e, 0), P.n_elem - 1);
            const double fd = rx_directivity(P, -d.z);
            int txl;
            uint32_t rid;
            ray_of(a, ci, &txl, &rid);
            Deposit dp;
            n_dep += fd > 0.0;
            if (fd > 0.0 && make_deposit((uint32_t)((a.tx_base + txl) * P.n_elem + e), P.n_t, P.fs, th, wh * fd, &dp))
              add_deposit(a.h, P.n_t, dp, a.hist_scale, a.hist_over);
          }
        }
      } else if (h.kind != kHitNone && k <= B) {
        if (kDeposit) ++n_int;
        int txl;
        uint32_t rid;
        ray_of(a, ci, &txl, &rid);
        const Step st = step_at(S, o, d, t, w, region, h);
        t = st.tp;
        w = st.watt;
        const Draw v = draw(a.seed, rid, a.tx.id[txl], (uint32_t)k);
        const double p_spec = (1.0 - st.sf.kd) * st.f.RE;
        bool alive = true;
        if (v.u0 < p_spec) {
          if (st.sf.rho > 0.0) {
            const Glossy gl = glossy_reflect(d, st.f, st.sf.rho, v.u1, v.u2);
            d = gl.dir;
            w *= st.f.Ar / st.f.RE * gl.g;
            alive = gl.ok;
          } else {
            d = d + st.f.nr * (2.0 * st.f.ci);
            w *= st.f.Ar / st.f.RE;
          }
          delta = true;
        } else if (v.u0 < st.f.RE) {
          const d3 nn = st.f.nr;
          const double sg = nn.z >= 0.0 ? 1.0 : -1.0;
          const double aa = -1.0 / (sg + nn.z);
          const double bb = nn.x * nn.y * aa;
          const d3 b1{1.0 + sg * nn.x * nn.x * aa, sg * bb, -sg * nn.x};
          const d3 b2{bb, sg + nn.y * nn.y * aa, -nn.y};
          const double phi = 2.0 * kPi * v.u1, rr = sqrt(v.u2);
          const SinCos sc = sincos_ool(phi);
          d = b1 * (rr * sc.c) + b2 * (rr * sc.s) + nn * sqrt(1.0 - v.u2);
          w *= st.f.Ar / st.f.RE;
          delta = false;
        } else {
          const double eta = S.c[st.sf.other] / S.c[region];
          d = d * eta + st.f.nr * (eta * st.f.ci - st.f.ct);
          w *= st.f.At / (1.0 - st.f.RE);
          region = st.sf.other;
          delta = true;
        }
        o = st.x;
        a.stk.last[ci] = k;
        keep = alive;
        diffuse = st.sf.kd > 0.0;
        if (diffuse && a.sort.keys > 0)
          skey = a.sort.key(st.x.x, st.x.z, min((int)(v.u3 * (double)P.n_elem), P.n_elem - 1));
      }
    }
    const Slots sl = block_append2(keep, diffuse, &a.counts[k], scan);
    const long slot = sl.a;
    if (sl.b >= 0) {
      a.stk.queue[(long)(k - 1) * cap + sl.b] = ci;
      if (a.sort.keys > 0) {
        const uint32_t rank = atomicAdd(a.sort_count + (long)(k - 1) * a.sort.keys + skey, 1u);
        a.stk.sort_kr[(long)(k - 1) * cap + sl.b] = make_uint2(skey, rank);
      }
    }
    if (slot >= 0) {
      a.qout.ox[slot] = o.x; a.qout.oy[slot] = o.y; a.qout.oz[slot] = o.z;
      a.qout.dx[slot] = d.x; a.qout.dy[slot] = d.y; a.qout.dz[slot] = d.z;
      a.qout.t[slot] = t; a.qout.w[slot] = w;
      a.qout.rid[slot] = ci;
      a.qout.meta[slot] = (uint32_t)region | ((uint32_t)delta << 8);
    }
  }
  if (kDeposit && a.counters) flush_counters(a.counters, n_seg, 0, n_dep, n_int, 0);
}

// Phase 2 (one thread per queued interaction): the secondary ray towards
// the element the interaction picked, with its parameter adjoints, and the
// adjoints of its inputs (x, n_r, A_r, w_att, t') kept for phase 3.
// Exclusive prefix over the diffuse interactions of the steps (high halves
// of the counts): step k's entries are number queue_begin[k - 1] onwards.
__global__ void k_replay_prefix(ReplayArgs a) {
  if (threadIdx.x != 0) return;
  unsigned long long run = 0;
  a.stk.queue_begin[0] = 0;
  for (int k = 1; k <= a.max_bounces; ++k) {
    run += a.counts[k] >> 32;
    a.stk.queue_begin[k] = run;
  }
}

// Queued interaction q (step k, slot q - queue_begin[k - 1]) to its place in
// key order: the offset of (k, key) plus its rank.
__global__ __launch_bounds__(256) void k_replay_sort_scatter(ReplayArgs a) {
  const int B = a.max_bounces;
  const long n_q = B > 0 ? (long)a.stk.queue_begin[B] : 0;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n_q; q += (long)gridDim.x * blockDim.x) {
    int k = 1, hi = B;
    while (k < hi) {
      const int mid = (k + hi + 1) >> 1;
      if ((long)a.stk.queue_begin[mid - 1] <= q) k = mid; else hi = mid - 1;
    }
    const long e = (long)(k - 1) * a.cap + (q - (long)a.stk.queue_begin[k - 1]);
    const uint2 kr = a.stk.sort_kr[e];
    a.stk.sort_q[a.sort_count[(long)(k - 1) * a.sort.keys + kr.x] + kr.y] = a.stk.queue[e];
  }
}

// Receiver segments of a recorded forward (one thread per queued diffuse
// interaction, in key order): the secondary ray rebuilt from the step record
// and its draw, weighted as the bounce kernel weights it, marched and
// deposited as the secondary kernel does, so that the histogram is the plain
// forward's.
template <bool kMeshes>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_replay_deposit(ReplayArgs a) {
  const int B = a.max_bounces;
  const long n_q = B > 0 ? (long)a.stk.queue_begin[B] : 0;
  if ((long)blockIdx.x * blockDim.x >= n_q) return;
  __shared__ SceneLDS S;
  extern __shared__ int bvh_stack[];
  load_scene(S, a.scene);
  int* stk = bvh_stack + threadIdx.x;
  const ProbeView& P = a.probe;
  const long cap = a.cap;
  uint32_t n_seg = 0, n_dep = 0, n_rays = 0;   // event counters, as the secondary kernel counts them
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n_q; q += (long)gridDim.x * blockDim.x) {
    int k = 1, hi = B;
    while (k < hi) {
      const int mid = (k + hi + 1) >> 1;
      if ((long)a.stk.queue_begin[mid - 1] <= q) k = mid; else hi = mid - 1;
    }
    const uint32_t i = a.sort.keys > 0 ? a.stk.sort_q[q]
                                       : a.stk.queue[(long)(k - 1) * cap + (q - (long)a.stk.queue_begin[k - 1])];
    int txl;
    uint32_t rid;
    ray_of(a, i, &txl, &rid);
    const StepRec R = a.stk.rec[(long)(k - 1) * cap + i];
    const int reg = R.meta & 0xFF;
    const Hit h{(int)(R.meta >> 12), R.hidx, R.L};
    const Step st = step_at(S, d3{R.ox, R.oy, R.oz}, d3{R.dx, R.dy, R.dz}, R.t, R.w, reg, h);
    const Draw v = draw(a.seed, rid, a.tx.id[txl], (uint32_t)k);
    const int e2 = min((int)(v.u3 * (double)P.n_elem), P.n_elem - 1);
    const d3 dv = d3{elem_x(P, e2), 0.0, 0.0} - st.x;
    const double r = sqrt(dot(dv, dv));
    const d3 we = dv * (1.0 / r);
    const MarchRecs& M = a.march;
    const bool keep = q < M.cap;   // its march is recorded
    const double cos_o = dot(st.f.nr, we);
    const double cos_el = -we.z;
    const double fd = cos_o > 0.0 ? rx_directivity(P, cos_el) : 0.0;
    if (!(cos_o > 0.0) || fd == 0.0) {
      if (keep) M.nstate[q] = 0u;
      continue;
    }
    ++n_rays;
    double amp = st.watt * st.f.Ar * (st.sf.kd / kPi) * cos_o * (P.elem_w * P.elem_h * cos_el / (r * r)) *
                 (double)P.n_elem * fd;
    const March mr = receiver_march<kMeshes>(S, st.x, we, r, reg, st.tp, stk,
                                             [&](int j, double sj, int hw, const Surface&, const Coef&) {
                                               if (keep && j < kMarchLegs) {
                                                 M.s[j * M.cap + q] = sj;
                                                 M.h[j * M.cap + q] = hw;
                                               }
                                             });
    if (keep) {
      M.tof[q] = mr.tof;
      M.att[q] = mr.att;
      M.trans[q] = mr.trans;
      M.nstate[q] = (uint32_t)mr.crossings << 2 | (mr.reached ? 2u : 1u);
    }
    n_seg += mr.reached ? mr.crossings + 1 : mr.crossings;   // one segment per leg
    if (!mr.reached) continue;
    ++n_dep;
    amp *= mr.trans;
    amp *= exp_ool(-mr.att);
    Deposit dp;
    if (make_deposit((uint32_t)((a.tx_base + txl) * P.n_elem + e2), P.n_t, P.fs, mr.tof, amp, &dp))
      add_deposit(a.h, P.n_t, dp, a.hist_scale, a.hist_over);
  }
  if (a.counters) flush_counters(a.counters, 0, n_seg, n_dep, 0, n_rays);
}

// Acquisition-parameter adjoints of one block (the steering angles of the
// launch group's transmits, then c_ref, the pitch and f0) in LDS accumulators
// after the gradient copies (when the call asks for them), added to the global
// accumulators of a.acq_sum (entry tx_base + j for transmit j) once per block.
__device__ __forceinline__ int acq_words(const ReplayArgs& a) { return a.g_acq ? (a.tx.n + 3) * kSumWords : 0; }

__device__ __forceinline__ void acq_flush(const ReplayArgs& a, const unsigned long long* acq) {
  if (!a.g_acq) return;
  for (int j = threadIdx.x; j < acq_words(a); j += blockDim.x) {
    const unsigned long long v = acq[j];
    const int e = j / kSumWords, w = j % kSumWords;
    const int g = e < a.tx.n ? a.tx_base + e : a.n_tx_total + (e - a.tx.n);
    if (v) atomicAdd(a.acq_sum + (long)g * kSumWords + w, v);
  }
}

template <bool kMeshes>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMeshes ? 2 : 3, 8))) void k_replay_secondary(ReplayArgs a) {
  const int B = a.max_bounces;
  const long n_q = B > 0 ? (long)a.stk.queue_begin[B] : 0;
  if ((long)blockIdx.x * blockDim.x >= n_q) return;
  __shared__ SceneLDS S;
  // gradient accumulators (grad_copies copies), acquisition accumulators,
  // crossing caches, hierarchy stacks
  extern __shared__ unsigned long long gsh[];
  load_scene(S, a.scene);
  const int gw = a.grad_copies * grad_words(a.n_grad);
  unsigned long long* acq = gsh + gw;
  words_clear(gsh, gw + acq_words(a));
  __syncthreads();
  constexpr int kVn = 1 << kVhBitsSecondary;
  uint32_t* hk = (uint32_t*)(acq + acq_words(a));   // vertex sum table (mesh scenes)
  unsigned long long* hw = (unsigned long long*)(hk + kVn);
  if (kMeshes) {
    vh_clear(hk, hw, kVn);
    __syncthreads();
  }
  double* legs = kMeshes ? (double*)(hw + 2 * kVn) : (double*)(acq + acq_words(a));
  double* leg_t = legs + threadIdx.x;
  int* leg_h = (int*)(legs + kLegCache * blockDim.x) + threadIdx.x;
  int* stk = leg_h + kLegCache * blockDim.x;
  GradAcc G{gsh + (threadIdx.x % a.grad_copies) * grad_words(a.n_grad), a.scene.n_regions, a.scene.n_planes,
            a.scene.n_spheres, a.scene.n_cylinders, a.scene.np_per_m, a.scene.vnormal,
            a.vadj + (long)(blockIdx.x % kVadjCopies) * a.vadj_stride * kSumWords, a.vadj_stride};
  if (kMeshes) {
    G.hk = hk;
    G.hw = hw;
    G.vh_bits = kVhBitsSecondary;
  }
  const ProbeView& P = a.probe;
  const long cap = a.cap;
  // block-uniform loop: the vertex table is flushed after each pass of the block
  for (long qb = (long)blockIdx.x * blockDim.x; qb < n_q; qb += (long)gridDim.x * blockDim.x) {
    const long q = qb + threadIdx.x;
    if (q < n_q) {
      // the step k with queue_begin[k - 1] <= q < queue_begin[k]
      int k = 1, hi = B;
      while (k < hi) {
        const int mid = (k + hi + 1) >> 1;
        if ((long)a.stk.queue_begin[mid - 1] <= q) k = mid; else hi = mid - 1;
      }
      const uint32_t i = a.sort.keys > 0 ? a.stk.sort_q[q]
                                         : a.stk.queue[(long)(k - 1) * cap + (q - (long)a.stk.queue_begin[k - 1])];
      const long at = (long)(k - 1) * cap + i;
      int txl;
      uint32_t rid;
      ray_of(a, i, &txl, &rid);
      const StepRec R = a.stk.rec[at];
      const d3 o{R.ox, R.oy, R.oz};
      const d3 d{R.dx, R.dy, R.dz};
      const uint32_t meta = R.meta;
      const int reg = meta & 0xFF;
      const Hit h{(int)(meta >> 12), R.hidx, R.L};
      const Step st = step_at(S, o, d, R.t, R.w, reg, h);
      const Draw v = draw(a.seed, rid, a.tx.id[txl], (uint32_t)k);
      const int e2 = min((int)(v.u3 * (double)P.n_elem), P.n_elem - 1);
      ReplayCtx C{S, P, a.gh, a.gh_f0, (long)(a.tx_base + txl) * P.n_elem, G, stk, leg_t, leg_h,
                  a.march, q < a.march.cap ? q : -1L};
      d3 xb{0, 0, 0}, nrb{0, 0, 0};
      double Ab = 0.0, wb = 0.0, tb = 0.0, xeb = 0.0, f0b = 0.0;
      secondary_backward<kMeshes>(C, reg, st.x, st.f, st.sf.kd, st.watt, st.tp, e2, xb, nrb, Ab, wb, tb, xeb, f0b);
      a.stk.adj[at] = StepAdj{xb.x, xb.y, xb.z, nrb.x, nrb.y, nrb.z, Ab, wb, tb, 0.0};
      // x_e = (e - (N - 1)/2) pitch
      if (a.g_acq) {
        sum_add(acq + (a.tx.n + 1) * kSumWords, xeb * ((double)e2 - 0.5 * (double)(P.n_elem - 1)));
        sum_add(acq + (a.tx.n + 2) * kSumWords, f0b);
      }
    }
    if (kMeshes) vh_flush(hk, hw, G.vadj, G.vstride, kVn);
  }
  __syncthreads();
  grad_flush(gsh, a.n_grad, a.grad_copies, a.g_sum);
  acq_flush(a, acq);
}

// Phase 3 (one thread per ray): the reverse sweep over the kept steps, with
// the secondary-ray adjoints of phase 2 added at their interactions; no
// intersection queries.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_replay_reverse(ReplayArgs a, long n) {
  if ((long)blockIdx.x * blockDim.x >= n) return;
  __shared__ SceneLDS S;
  extern __shared__ unsigned long long gsh[];   // gradient accumulators (grad_copies copies), acquisition accumulators
  load_scene(S, a.scene);
  const int gw = a.grad_copies * grad_words(a.n_grad);
  unsigned long long* acq = gsh + gw;
  words_clear(gsh, gw + acq_words(a));
  constexpr int kVn = 1 << kVhBitsReverse;
  uint32_t* hk = (uint32_t*)(acq + acq_words(a));   // vertex sum table (mesh scenes)
  unsigned long long* hw = (unsigned long long*)(hk + kVn);
  const bool vh = a.scene.n_meshes > 0;
  if (vh) vh_clear(hk, hw, kVn);
  __syncthreads();
  GradAcc G{gsh + (threadIdx.x % a.grad_copies) * grad_words(a.n_grad), a.scene.n_regions, a.scene.n_planes,
            a.scene.n_spheres, a.scene.n_cylinders, a.scene.np_per_m, a.scene.vnormal,
            a.vadj + (long)(blockIdx.x % kVadjCopies) * a.vadj_stride * kSumWords, a.vadj_stride};
  if (vh) {
    G.hk = hk;
    G.hw = hw;
    G.vh_bits = kVhBitsReverse;
  }
  const ProbeView& P = a.probe;
  const long cap = a.cap;
  // block-uniform loop: the vertex table is flushed after each pass of the block
  for (long base = (long)blockIdx.x * blockDim.x; base < n; base += (long)gridDim.x * blockDim.x) {
    const long i = base + threadIdx.x;
    if (i < n) {
      int txl;
      uint32_t rid;
      ray_of(a, i, &txl, &rid);
      const uint32_t tx_id = a.tx.id[txl];
      const long row_base = (long)(a.tx_base + txl) * P.n_elem;
      d3 ob{0, 0, 0}, db{0, 0, 0};
      double tb = 0.0, wb = 0.0;
      for (int k = a.stk.last[i]; k >= 1; --k) {
        const long at = (long)(k - 1) * cap + i;
        const StepRec R = a.stk.rec[at];
        const uint32_t meta = R.meta;
        const d3 o0{R.ox, R.oy, R.oz};
        const d3 d0{R.dx, R.dy, R.dz};
        const double t0 = R.t, w0 = R.w;
        const int reg = meta & 0xFF;
        const bool dl = (meta >> 8) & 1u;
        const Hit h{(int)(meta >> 12), R.hidx, R.L};
        const Step st = step_at(S, o0, d0, t0, w0, reg, h);
        const double L = st.L, c1 = S.c[reg], ar = S.a[reg];
        const double watt = st.watt;
        const d3 x = st.x;
        d3 xb{0, 0, 0}, d0b{0, 0, 0};
        TriAdj ta;   // the hit triangle's adjoints from the normal and the distance
        double tpb = 0.0, wattb = 0.0;
        if (h.kind == kHitArray) {
          const double half = 0.5 * (double)P.n_elem * P.pitch;
          if (dl && fabs(x.x) < half && fabs(x.y) < 0.5 * P.elem_h) {
            int e = (int)floor((x.x + half) / P.pitch);
            e = min(max(e, 0), P.n_elem - 1);
            const double fd = rx_directivity(P, -d0.z);
            if (fd > 0.0) {
              double ga, gt;
              tent_adjoint(a.gh + (row_base + e) * (long)P.n_t, P.n_t, P.fs, st.tp, watt * fd, &ga, &gt);
              if (a.gh_f0) {
                double gf, unused;
                tent_adjoint(a.gh_f0 + (row_base + e) * (long)P.n_t, P.n_t, P.fs, st.tp, 0.0, &gf, &unused);
                sum_add(acq + (a.tx.n + 2) * kSumWords, gf * watt * fd);
              }
              wattb += ga * fd;
              d0b.z -= ga * watt * rx_directivity_deriv(P, -d0.z);
              tpb += gt;
            }
          }
        } else {
          const Surface sf = st.sf;
          const Coef f = st.f;
          const int r2 = sf.other;
          const Draw v = draw(a.seed, rid, tx_id, (uint32_t)k);
          const double eta = S.c[r2] / c1;
          xb = ob;
          tpb = tb;
          d3 nrb{0, 0, 0};
          double cib = 0.0, ctb = 0.0, etab = 0.0, Ab = 0.0;
          const double p_spec = (1.0 - sf.kd) * f.RE;
          if (v.u0 < p_spec) {
            // d' = d - 2 (d.m) m about the GGX microfacet m(n_r, rho), w' = watt
            // Ar / R_E g. Taken in this form also at rho = 0, where the forward
            // mirrored about n_r: the values agree and dL/drho is kept.
            const d3 nn = f.nr;
            const Frame fr = frame_of(nn);
            const double rho = sf.rho;
            const double kap = sqrt(v.u1 / (1.0 - v.u1));
            const double th = rho * kap;
            const double lz = 1.0 / sqrt(1.0 + th * th);
            const double sh = th * lz;
            const double phi = 2.0 * kPi * v.u2;
            const SinCos scp = sincos_ool(phi);
            const double cph = scp.c, sph = scp.s;
            const double lx = sh * cph, ly = sh * sph;
            const d3 m = fr.b1 * lx + fr.b2 * ly + nn * lz;
            const double wh = dot(d0, m);
            const d3 dout = d0 - m * (2.0 * wh);
            const double co = dot(nn, dout);
            if (wh < 0.0 && co > 0.0) {   // else the path ended here: nothing flows back
              const double g1i = smith_g1(f.ci, rho), g1o = smith_g1(co, rho);
              const double q = f.ci * lz, g = g1i * g1o * (-wh) / q;
              wattb += wb * f.Ar / f.RE * g;
              Ab += wb * watt / f.RE * g;
              const double gb = wb * watt * f.Ar / f.RE;
              double rho_b = 0.0, co_b = 0.0, lz_b = -gb * g / lz;
              cib += -gb * g / f.ci;
              smith_g1_vjp(f.ci, rho, gb * g1o * (-wh) / q, &cib, &rho_b);
              smith_g1_vjp(co, rho, gb * g1i * (-wh) / q, &co_b, &rho_b);
              const double im_b = gb * g1i * g1o / q;            // of -wh
              const d3 ob = db + nn * co_b;                      // co = n_r . d'
              nrb = nrb + dout * co_b;
              d0b = d0b + ob;
              const double wh_b = -2.0 * dot(m, ob) - im_b;
              const d3 mb = ob * (-2.0 * wh) + d0 * wh_b;
              d0b = d0b + m * wh_b;
              nrb = nrb + frame_vjp(nn, lx, ly, lz, mb);
              lz_b += dot(nn, mb);
              const double sh_b = dot(fr.b1, mb) * cph + dot(fr.b2, mb) * sph;
              const double lz3 = lz * lz * lz;
              rho_b += sh_b * kap * lz3 - lz_b * rho * kap * kap * lz3;
              G.rough(h.kind, h.kind == kHitMesh ? S.tri[h.index].w : h.index, rho_b);
            }
          } else if (v.u0 < f.RE) {     // d' = lx b1(nr) + ly b2(nr) + lz nr
            const double phi = 2.0 * kPi * v.u1, rr = sqrt(v.u2);
            const SinCos sc = sincos_ool(phi);
            const double lx = rr * sc.c, ly = rr * sc.s, lz = sqrt(1.0 - v.u2);
            nrb = nrb + frame_vjp(f.nr, lx, ly, lz, db);
            wattb += wb * f.Ar / f.RE;
            Ab += wb * watt / f.RE;
          } else {                      // d' = eta d + (eta ci - ct) nr, w' = watt At / (1 - R_E)
            const double dn = dot(db, f.nr);
            d0b = d0b + db * eta;
            etab += dot(db, d0) + f.ci * dn;
            cib += eta * dn;
            ctb -= dn;
            nrb = nrb + db * (eta * f.ci - f.ct);
            wattb += wb * f.At / (1.0 - f.RE);
            Ab += wb * watt / (1.0 - f.RE);
          }
          if (sf.kd > 0.0) {   // adjoints of the secondary ray's inputs (phase 2)
            const StepAdj Q = a.stk.adj[at];
            xb = xb + d3{Q.xb, Q.yb, Q.zb};
            nrb = nrb + d3{Q.nxb, Q.nyb, Q.nzb};
            Ab += Q.Ab;
            wattb += Q.wb;
            tpb += Q.tb;
          }
          cib += interface_backward(f, eta, reg, r2, S.Z[reg], S.Z[r2], c1, Ab, ctb, etab, G);
          // ci = -nr . d
          nrb = nrb - d0 * cib;
          d0b = d0b - f.nr * cib;
          const double sgn = dot(sf.n, d0) > 0.0 ? -1.0 : 1.0;
          normal_backward(S, h.kind, h.index, sf.n, nrb * sgn, xb, G, ta);
        }
        // t' = t + L / c, w_att = w exp(-a L), x = o + d L, L = distance(o, d)
        const double Lb = tpb / c1 - wattb * watt * ar + dot(xb, d0);
        G.c(reg, -tpb * L / (c1 * c1));
        G.a(reg, -wattb * watt * L);
        d3 o0b = xb;
        d0b = d0b + xb * L;
        const double sig = h.kind == kHitSphere     ? primary_root(S, h.index, o0, d0)
                         : h.kind == kHitCylinder ? cylinder_root(S, h.index, o0, d0)
                                                  : -1.0;
        distance_backward(S, h.kind, h.index, sig, o0, d0, L, Lb, o0b, d0b, G, ta);
        if (h.kind == kHitMesh) tri_nu_backward(S, h.index, ta.nub, ta.p0b, G);
        ob = o0b;
        db = d0b;
        tb = tpb;
        wb = wattb * st.E;
      }
      if (a.g_acq) {
        // the emitted state: o = (x_e + (u0 - 1/2) w_el, (u1 - 1/2) h_el, 0),
        // d = (sin th, 0, cos th), t = o_x sin th / c_ref, w = cos th / n, with
        // x_e = (e - (N - 1)/2) pitch
        const int e = (int)(rid / (uint32_t)a.rays_per_elem);
        const Draw u = draw(a.seed, rid, tx_id, 0);
        const double de = (double)e - 0.5 * (double)(P.n_elem - 1);
        const double ox = elem_x(P, e) + (u.u0 - 0.5) * P.elem_w;
        const double sa = a.tx.sin_a[txl], ca = a.tx.cos_a[txl];
        const double thb = db.x * ca - db.z * sa + tb * ox * ca / P.c_ref - wb * sa / (double)a.rays_per_elem;
        sum_add(acq + txl * kSumWords, thb);
        sum_add(acq + a.tx.n * kSumWords, -tb * ox * sa / (P.c_ref * P.c_ref));
        sum_add(acq + (a.tx.n + 1) * kSumWords, (ob.x + tb * sa / P.c_ref) * de);
      }
    }
    if (vh) vh_flush(hk, hw, G.vadj, G.vstride, kVn);
  }
  __syncthreads();
  grad_flush(gsh, a.n_grad, a.grad_copies, a.g_sum);
  acq_flush(a, acq);
}

// vval[v] = the total of vertex v's adjoint sums over the kVadjCopies copies
// (their words added first, then read out).
__global__ __launch_bounds__(256) void k_vertex_values(const unsigned long long* __restrict__ vadj, long stride,
                                                       long n_v, double* __restrict__ vval) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_v) return;
  unsigned long long w[kSumWords];
#pragma unroll
  for (int k = 0; k < kSumWords; ++k) w[k] = 0ull;
  for (int c = 0; c < kVadjCopies; ++c) {
    const unsigned long long* p = vadj + (long)c * stride * kSumWords + v;
#pragma unroll
    for (int k = 0; k < kSumWords; ++k) w[k] += p[k * stride];
  }
  vval[v] = sum_value(w);
}

// g_theta[q(m, j)] += sum over the vertices v of mesh m of vval[v] phi_j(v):
// one block per (mesh, basis function), vertices of mesh m in
// [vbeg[m], vbeg[m + 1]), summed in a fixed tree.
__global__ __launch_bounds__(256) void k_basis_gather(const double* __restrict__ vval,
                                                      const double* __restrict__ vbasis,
                                                      const long* __restrict__ vbeg, int n_basis,
                                                      double* __restrict__ g_q) {
  const int m = blockIdx.x / n_basis, j = blockIdx.x % n_basis;
  double acc = 0.0;
  for (long v = vbeg[m] + threadIdx.x; v < vbeg[m + 1]; v += blockDim.x) acc += vval[v] * vbasis[v * n_basis + j];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g_q[blockIdx.x] += red[0];   // this block is the entry's only writer
}

// g_theta[j] += the total of accumulator j, j < n_grad; with g_acq, also
// g_acq[i] += the total of acquisition accumulator i, i < n_acq, and the f0
// entry (index f0_at) takes sum_r theta[3 r + 2] dL/dalpha_r * inv_f0 besides
// (every region's amplitude attenuation alpha_r np_per_m grows in proportion
// to f0). One block; every entry is read out in a fixed order.
__global__ __launch_bounds__(256) void k_grad_finish(const unsigned long long* __restrict__ g_sum, int n_grad,
                                                     double* __restrict__ g_theta,
                                                     const unsigned long long* __restrict__ acq_sum, int n_acq,
                                                     double* __restrict__ g_acq, int f0_at,
                                                     const double* __restrict__ theta, int n_regions,
                                                     double inv_f0) {
  for (int j = threadIdx.x; j < n_grad; j += blockDim.x) g_theta[j] += sum_value(g_sum + (long)j * kSumWords);
  if (!g_acq) return;
  for (int i = threadIdx.x; i < n_acq; i += blockDim.x) {
    double v = sum_value(acq_sum + (long)i * kSumWords);
    if (i == f0_at) {
      double att = 0.0;
      for (int r = 0; r < n_regions && 3 * r + 2 < n_grad; ++r)
        att += sum_value(g_sum + (long)(3 * r + 2) * kSumWords) * theta[3 * r + 2];
      v += att * inv_f0;
    }
    g_acq[i] += v;
  }
}

namespace {
unsigned replay_grid(long n, long cap = kMaxReplayBlocks) {
  const long b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}
// the forward phase keeps no gradient sums, so its grid may be larger
constexpr long kMaxReplayForwardBlocks = 8192;
size_t stack_lds(const ReplayArgs& a) {
  return a.scene.n_meshes > 0 ? (size_t)a.scene.stack_cap * 256 * sizeof(int) : 0;
}
size_t acq_lds(const ReplayArgs& a) { return a.g_acq ? (size_t)(a.tx.n + 3) * kSumWords * 8 : 0; }
// LDS of a block of 256 threads when `waves` of them share a SIMD: the
// gradient copies get what the rest leaves (at most 16 copies, at least one).
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr size_t kStaticLds = 8192;   // the scene copy and the kernels' own arrays, rounded up
int grad_copies_for(const ReplayArgs& a, int waves, size_t other) {
  const size_t budget = kLdsPerCU / waves;
  const size_t per = (size_t)a.n_grad * kSumWords * 8;
  int c = 16;
  while (c > 1 && kStaticLds + other + c * per > budget) c >>= 1;
  return c;
}
size_t grad_lds(const ReplayArgs& a) { return (size_t)a.grad_copies * a.n_grad * kSumWords * 8; }
}  // namespace

void launch_replay_forward(const ReplayArgs& a, int k, long n, hipStream_t s) {
  const bool m = a.scene.n_meshes > 0;
  const auto kern = a.h ? (m ? k_replay_forward<true, true> : k_replay_forward<false, true>)
                        : (m ? k_replay_forward<true, false> : k_replay_forward<false, false>);
  hipLaunchKernelGGL(kern, dim3(replay_grid(n, kMaxReplayForwardBlocks)), dim3(256), stack_lds(a), s, a, k, n);
}

void launch_replay_secondary(const ReplayArgs& a0, long max_entries, hipStream_t s) {
  ReplayArgs a = a0;
  const size_t legs = (size_t)kLegCache * 256 * (sizeof(double) + sizeof(int));
  const bool m = a.scene.n_meshes > 0;
  const size_t vhb = m ? vh_bytes(kVhBitsSecondary) : 0;
  a.grad_copies = grad_copies_for(a, m ? 2 : 3, acq_lds(a) + legs + stack_lds(a) + vhb);
  const auto kern = m ? k_replay_secondary<true> : k_replay_secondary<false>;
  hipLaunchKernelGGL(kern, dim3(replay_grid(max_entries)), dim3(256),
                     grad_lds(a) + acq_lds(a) + legs + stack_lds(a) + vhb, s, a);
}

void launch_replay_deposit(const ReplayArgs& a, long max_entries, hipStream_t s) {
  const auto kern = a.scene.n_meshes > 0 ? k_replay_deposit<true> : k_replay_deposit<false>;
  hipLaunchKernelGGL(kern, dim3(replay_grid(max_entries, kMaxReplayForwardBlocks)), dim3(256), stack_lds(a), s, a);
}

void launch_replay_prefix(const ReplayArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_replay_prefix, dim3(1), dim3(64), 0, s, a);
}

void launch_replay_sort(const ReplayArgs& a, long max_entries, hipStream_t s) {
  if (a.sort.keys <= 0 || a.max_bounces <= 0) return;
  launch_sort_offsets(a.sort_count, a.max_bounces * a.sort.keys, a.sort_part, s);
  hipLaunchKernelGGL(k_replay_sort_scatter, dim3(replay_grid(max_entries, kMaxReplayForwardBlocks)), dim3(256), 0,
                     s, a);
}

void launch_grad_finish(const unsigned long long* g_sum, int n_grad, double* g_theta,
                        const unsigned long long* acq_sum, int n_acq, double* g_acq, int f0_at,
                        const double* theta, int n_regions, double inv_f0, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(256), 0, s, g_sum, n_grad, g_theta, acq_sum, n_acq, g_acq, f0_at,
                     theta, n_regions, inv_f0);
}

void launch_replay_reverse(const ReplayArgs& a0, long n, hipStream_t s) {
  ReplayArgs a = a0;
  const size_t vhb = a.scene.n_meshes > 0 ? vh_bytes(kVhBitsReverse) : 0;
  a.grad_copies = grad_copies_for(a, 3, acq_lds(a) + vhb);
  hipLaunchKernelGGL(k_replay_reverse, dim3(replay_grid(n)), dim3(256), grad_lds(a) + acq_lds(a) + vhb, s, a, n);
}

void launch_basis_gather(const unsigned long long* vadj, long stride, long n_vertices, double* vval,
                         const double* vbasis, const long* vbeg, int n_meshes, int n_basis, double* g_q,
                         hipStream_t s) {
  if (n_meshes <= 0 || n_basis <= 0 || n_vertices <= 0) return;
  hipLaunchKernelGGL(k_vertex_values, dim3((unsigned)((n_vertices + 255) / 256)), dim3(256), 0, s, vadj, stride,
                     n_vertices, vval);
  hipLaunchKernelGGL(k_basis_gather, dim3(n_meshes * n_basis), dim3(256), 0, s, vval, vbasis, vbeg, n_basis, g_q);
}

}  // namespace usrt
