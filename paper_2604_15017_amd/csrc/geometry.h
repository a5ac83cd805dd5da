// Device geometry and interface physics shared by the forward transport and
// the replay backward, so that both take identical discrete decisions.
#pragma once

#include "common.h"

namespace usrt {

struct Hit { int kind; int index; double t; };

__device__ __forceinline__ d3 vtx(gptr<double> v, int i) {
  return d3{v[3 * i], v[3 * i + 1], v[3 * i + 2]};
}
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
  return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Ray against one fp32 child box (already padded outward by kBoxPad by the
// refit, which absorbs the rounding of the ray to fp32): with oi = o * (1/d)
// per axis, the slab distances are lo * (1/d) - oi, one fused multiply-add
// each; entry distance in *t0, culled beyond lim.
__device__ __forceinline__ bool slab(const float* lo, const float* hi, float oix, float oiy, float oiz,
                                     float ix, float iy, float iz, float lim, float* t0) {
  const float ax = fmaf(lo[0], ix, -oix), bx = fmaf(hi[0], ix, -oix);
  const float ay = fmaf(lo[1], iy, -oiy), by = fmaf(hi[1], iy, -oiy);
  const float az = fmaf(lo[2], iz, -oiz), bz = fmaf(hi[2], iz, -oiz);
  const float tmin = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
  const float tmax = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
  *t0 = tmin;
  return tmin <= tmax && tmin <= lim;
}

// The ray in the form the slab tests take: 1/d per axis (clamped away from
// infinity) and o * (1/d), in fp32.
struct SlabRay { float ix, iy, iz, oix, oiy, oiz; };
__device__ __forceinline__ SlabRay slab_ray(d3 o, d3 d) {
  SlabRay r;
  r.ix = fabs(d.x) > 1e-30 ? (float)(1.0 / d.x) : copysignf(1e30f, (float)d.x);
  r.iy = fabs(d.y) > 1e-30 ? (float)(1.0 / d.y) : copysignf(1e30f, (float)d.y);
  r.iz = fabs(d.z) > 1e-30 ? (float)(1.0 / d.z) : copysignf(1e30f, (float)d.z);
  r.oix = (float)o.x * r.ix;
  r.oiy = (float)o.y * r.iy;
  r.oiz = (float)o.z * r.iz;
  return r;
}

// Moller-Trumbore in fp64 on a leaf-order triangle record, edges included;
// distance or -1. No branches: every quantity is formed and one select keeps
// the distance (a zero determinant gives an infinite or NaN barycentric,
// which the range tests, written to fail on NaN, reject).
__device__ __forceinline__ double rec_distance(const TriRec r, d3 o, d3 d) {
  const d3 e1{r.e1[0], r.e1[1], r.e1[2]}, e2{r.e2[0], r.e2[1], r.e2[2]};
  const d3 sv = o - d3{r.p0[0], r.p0[1], r.p0[2]};
  const d3 pv = cross(d, e2);
  const double det = dot(e1, pv);
  const double inv = 1.0 / det;
  const double u = dot(sv, pv) * inv;
  const d3 qv = cross(sv, e1);
  const double v = dot(d, qv) * inv;
  const double t = dot(e2, qv) * inv;
  return (u >= 0.0 && u <= 1.0 && v >= 0.0 && u + v <= 1.0) ? t : -1.0;
}

// Four child boxes of node n against the ray, culled beyond lim, as sort
// keys ordered by entry distance: the distance's fp32 bits (non-negative, so
// they order as integers) with the two low bits replaced by the child's
// slot, sorted by a five-exchange network of integer min / max (children
// closer than four ulps keep slot order). A missed child keys at or above
// kMissKey, the bits of INFINITY.
constexpr uint32_t kMissKey = 0x7F800000u;
__device__ __forceinline__ void node_children(const BvhNode& n, const SlabRay& q, float lim, uint32_t* k) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float lo[3] = {n.lox[j], n.loy[j], n.loz[j]}, hi[3] = {n.hix[j], n.hiy[j], n.hiz[j]};
    float tj;
    const float t = slab(lo, hi, q.oix, q.oiy, q.oiz, q.ix, q.iy, q.iz, lim, &tj) ? tj : INFINITY;
    k[j] = (__float_as_uint(t) & 0x7FFFFFFCu) | (uint32_t)j;
  }
#define USRT_CX(a, b)                                   \
  {                                                     \
    const uint32_t lo_ = min(k[a], k[b]), hi_ = max(k[a], k[b]); \
    k[a] = lo_; k[b] = hi_;                             \
  }
  USRT_CX(0, 1) USRT_CX(2, 3) USRT_CX(0, 2) USRT_CX(1, 3) USRT_CX(1, 2)
#undef USRT_CX
}

// The child reference of a sort key.
__device__ __forceinline__ int child_of(const BvhNode& n, uint32_t key) {
  const bool odd = key & 1u;
  const int c01 = odd ? n.child[1] : n.child[0], c23 = odd ? n.child[3] : n.child[2];
  return key & 2u ? c23 : c01;
}

// Walk of the 4-wide hierarchy near child first. An inner node's four child
// boxes are tested against the ray in fp32 and the hit children ordered by
// entry distance: the nearest is visited next, the others pushed farthest
// first. The stack lives in LDS, interleaved across the block's threads
// (entry i of this thread at stk[i * kWalkBlock]); it holds at most three
// entries per inner level. The walk alternates two phases so that the lanes
// of a wave run one kind of work at a time (Aila and Laine, HPG 2009): inner
// nodes until every lane holds a leaf (a lane that meets a leaf sets it aside
// and keeps walking), then the leaves. cull() is the distance beyond which
// boxes are skipped; leaf(first, count) tests a leaf's triangles.
constexpr int kWalkDone = 0x7FFFFFFF;
constexpr int kWalkBlock = 256;   // threads per block of every kernel that walks (its stack LDS is sized so)

template <class Cull, class Leaf>
__device__ __forceinline__ void walk4(const SceneLDS& s, const SlabRay& q, int* stk, Cull cull, Leaf leaf) {
  constexpr int step = kWalkBlock;
  int sp = 0, cur = 0, pend = 0;   // pend: a leaf set aside (leaf references are negative), 0 if none
  for (;;) {
    while ((unsigned)cur < (unsigned)kWalkDone) {   // an inner node
      const float lim = cull() * 1.0001f + kBoxPad;
      const BvhNode node = gload(s.nodes + cur);
      uint32_t k[4];
      node_children(node, q, lim, k);
      if (k[0] < kMissKey) {
        // the build bounds the depth by stack_cap / 3, so the pushes always fit
        if (k[3] < kMissKey && sp < s.stack_cap) { stk[sp * step] = child_of(node, k[3]); ++sp; }
        if (k[2] < kMissKey && sp < s.stack_cap) { stk[sp * step] = child_of(node, k[2]); ++sp; }
        if (k[1] < kMissKey && sp < s.stack_cap) { stk[sp * step] = child_of(node, k[1]); ++sp; }
        cur = child_of(node, k[0]);
      } else {
        cur = sp > 0 ? stk[--sp * step] : kWalkDone;
      }
      if (cur < 0 && pend == 0) {   // set the leaf aside and walk on
        pend = cur;
        cur = sp > 0 ? stk[--sp * step] : kWalkDone;
      }
      if (__all(pend != 0)) break;
    }
    while (pend != 0) {
      leaf((~pend) >> 4, (~pend) & 15);
      pend = 0;
      if (cur < 0) {   // the next reference is a leaf too
        pend = cur;
        cur = sp > 0 ? stk[--sp * step] : kWalkDone;
      }
    }
    if (cur == kWalkDone) break;
  }
}

// Closest triangle in (kTMin, best): best and best_tri updated.
__device__ __forceinline__ void mesh_closest(const SceneLDS& s, d3 o, d3 d, double& best, int& best_tri,
                                             int* stk) {
  walk4(s, slab_ray(o, d), stk, [&]() { return (float)best; }, [&](int first, int cnt) {
    for (int i = first; i < first + cnt; ++i) {
      const double t = rec_distance(gload(s.trec + i), o, d);
      if (t > kTMin && t < best) { best = t; best_tri = i; }
    }
  });
}

// Closest surface along o + t d with kTMin < t < tmax among the planes, the
// spheres, the meshes and, when `with_array` and the ray moves up, the array
// face z = 0.
// kMeshes = false compiles the hierarchy walk out (scenes without meshes).
template <bool kMeshes = true>
__device__ __forceinline__ Hit closest_hit(const SceneLDS& s, d3 o, d3 d, bool with_array,
                                           int* stk, double tmax = INFINITY) {
  Hit h{kHitNone, -1, 0.0};
  double best = tmax;
  if (d.z != 0.0) {
    const double inv = 1.0 / d.z;
    for (int k = 0; k < s.n_planes; ++k) {
      const double t = (s.pd[k] - o.z) * inv;
      if (t > kTMin && t < best) { best = t; h = Hit{kHitPlane, k, t}; }
    }
    if (with_array && d.z < 0.0) {
      const double t = -o.z * inv;
      if (t > kTMin && t < best) { best = t; h = Hit{kHitArray, -1, t}; }
    }
  }
  for (int k = 0; k < s.n_spheres; ++k) {
    const d3 oc{o.x - s.sx[k], o.y - s.sy[k], o.z - s.sz[k]};
    const double b = dot(oc, d);
    const double disc = b * b - (dot(oc, oc) - s.sr[k] * s.sr[k]);
    if (disc < 0.0) continue;
    const double q = sqrt(disc);
    const double t1 = -b - q;
    const double t = t1 > kTMin ? t1 : -b + q;
    if (t > kTMin && t < best) { best = t; h = Hit{kHitSphere, k, t}; }
  }
  // cylinders along y: a t^2 + 2 b t + cc = 0 in the x-z plane
  const double ca = d.x * d.x + d.z * d.z;
  if (ca > 0.0) {
    for (int k = 0; k < s.n_cylinders; ++k) {
      const double ox = o.x - s.cx[k], oz = o.z - s.cz[k];
      const double b = ox * d.x + oz * d.z;
      const double disc = b * b - ca * (ox * ox + oz * oz - s.cr[k] * s.cr[k]);
      if (disc < 0.0) continue;
      const double q = sqrt(disc);
      const double t1 = (-b - q) / ca;
      const double t = t1 > kTMin ? t1 : (-b + q) / ca;
      if (t > kTMin && t < best) { best = t; h = Hit{kHitCylinder, k, t}; }
    }
  }
  if (kMeshes && s.n_meshes > 0) {
    int tri = -1;
    mesh_closest(s, o, d, best, tri, stk);
    if (tri >= 0) h = Hit{kHitMesh, tri, best};
  }
  return h;
}

// Upper bound on the legs of a straight receiver segment: each plane is
// crossed once, each sphere twice, each closed mesh a few times (a segment
// that needs more is treated as blocked).
constexpr int kMeshLegs = 16;
__device__ __forceinline__ int max_legs(const SceneLDS& s) {
  return s.n_planes + 2 * s.n_spheres + 2 * s.n_cylinders + kMeshLegs * s.n_meshes + 1;
}

// Crossings of a straight segment x + s w, nearest first. A receiver segment
// is walked once for several crossings instead of once per leg: the walk keeps
// the kSegHits nearest surfaces with lo + kTMin < s < hi (every plane,
// sphere and cylinder crossing and every triangle hit) and culls boxes beyond
// the farthest kept one once the list is full. A full list may have dropped
// farther crossings; the caller then walks again from its last crossing.
// With lo the last crossing taken, a leg from it needs s > lo + kTMin, the
// same guard a per-leg closest-hit query from that point applies.
constexpr int kSegHits = 6;
struct SegHits {
  double s[kSegHits];   // ascending; unused entries hold +infinity
  int h[kSegHits];      // kind << 28 | index
  int n;
};

// Inserts s after the kept entries not greater than it, the last entry
// dropping out (nothing changes when the list is full and s is not below its
// last entry); selects only, no branches.
__device__ __forceinline__ void seg_insert(SegHits& L, double s, int h) {
#pragma unroll
  for (int j = kSegHits - 1; j > 0; --j) {
    const bool shift = s < L.s[j - 1], here = s < L.s[j];
    L.s[j] = shift ? L.s[j - 1] : here ? s : L.s[j];
    L.h[j] = shift ? L.h[j - 1] : here ? h : L.h[j];
  }
  const bool first = s < L.s[0];
  L.s[0] = first ? s : L.s[0];
  L.h[0] = first ? h : L.h[0];
  L.n = min(L.n + 1, kSegHits);
}

__device__ __forceinline__ double seg_cull(const SegHits& L, double hi) {
  return L.n == kSegHits ? L.s[kSegHits - 1] : hi;
}

template <bool kMeshes>
__device__ __forceinline__ SegHits segment_hits(const SceneLDS& s, d3 x, d3 w, double lo, double hi,
                                                int* stk) {
  SegHits L;
#pragma unroll
  for (int j = 0; j < kSegHits; ++j) { L.s[j] = INFINITY; L.h[j] = 0; }
  L.n = 0;
  const double smin = lo + kTMin;
  if (w.z != 0.0) {
    const double inv = 1.0 / w.z;
    for (int k = 0; k < s.n_planes; ++k) {
      const double t = (s.pd[k] - x.z) * inv;
      if (t > smin && t < hi) seg_insert(L, t, (kHitPlane << 28) | k);
    }
  }
  for (int k = 0; k < s.n_spheres; ++k) {
    const d3 oc{x.x - s.sx[k], x.y - s.sy[k], x.z - s.sz[k]};
    const double b = dot(oc, w);
    const double disc = b * b - (dot(oc, oc) - s.sr[k] * s.sr[k]);
    if (disc < 0.0) continue;
    const double q = sqrt(disc);
    const double t1 = -b - q, t2 = -b + q;
    if (t1 > smin && t1 < hi) seg_insert(L, t1, (kHitSphere << 28) | k);
    if (t2 > smin && t2 < hi) seg_insert(L, t2, (kHitSphere << 28) | k);
  }
  const double ca = w.x * w.x + w.z * w.z;
  if (ca > 0.0) {
    for (int k = 0; k < s.n_cylinders; ++k) {
      const double ox = x.x - s.cx[k], oz = x.z - s.cz[k];
      const double b = ox * w.x + oz * w.z;
      const double disc = b * b - ca * (ox * ox + oz * oz - s.cr[k] * s.cr[k]);
      if (disc < 0.0) continue;
      const double q = sqrt(disc);
      const double t1 = (-b - q) / ca, t2 = (-b + q) / ca;
      if (t1 > smin && t1 < hi) seg_insert(L, t1, (kHitCylinder << 28) | k);
      if (t2 > smin && t2 < hi) seg_insert(L, t2, (kHitCylinder << 28) | k);
    }
  }
  if (kMeshes && s.n_meshes > 0) {
    walk4(s, slab_ray(x, w), stk, [&]() { return (float)seg_cull(L, hi); }, [&](int first, int cnt) {
      for (int i = first; i < first + cnt; ++i) {
        const double t = rec_distance(gload(s.trec + i), x, w);
        if (t > smin && t < seg_cull(L, hi)) seg_insert(L, t, (kHitMesh << 28) | i);
      }
    });
  }
  return L;
}

// Unit face normal of leaf-order triangle i, from the current geometry.
__device__ __forceinline__ d3 tri_normal(const SceneLDS& s, int i) {
  const TriRec r = gload(s.trec + i);
  const d3 nu = cross(d3{r.e1[0], r.e1[1], r.e1[2]}, d3{r.e2[0], r.e2[1], r.e2[2]});
  return nu * (1.0 / sqrt(dot(nu, nu)));
}

struct Surface { d3 n; int other; double kd, rho; };

__device__ __forceinline__ Surface surface_of(const SceneLDS& s, const Hit& h, d3 x, int region) {
  Surface f;
  if (h.kind == kHitPlane) {
    f.n = d3{0.0, 0.0, 1.0};
    f.other = region == s.pr[h.index][0] ? s.pr[h.index][1] : s.pr[h.index][0];
    f.kd = s.pkd[h.index];
    f.rho = s.prho[h.index];
  } else if (h.kind == kHitSphere) {
    const double ir = 1.0 / s.sr[h.index];
    f.n = d3{(x.x - s.sx[h.index]) * ir, (x.y - s.sy[h.index]) * ir, (x.z - s.sz[h.index]) * ir};
    f.other = region == s.sreg[h.index][0] ? s.sreg[h.index][1] : s.sreg[h.index][0];
    f.kd = s.skd[h.index];
    f.rho = s.srho[h.index];
  } else if (h.kind == kHitCylinder) {
    const double ir = 1.0 / s.cr[h.index];
    f.n = d3{(x.x - s.cx[h.index]) * ir, 0.0, (x.z - s.cz[h.index]) * ir};
    f.other = region == s.creg[h.index][0] ? s.creg[h.index][1] : s.creg[h.index][0];
    f.kd = s.ckd[h.index];
    f.rho = s.crho[h.index];
  } else {
    const int m = s.tri[h.index].w;
    f.n = tri_normal(s, h.index);
    f.other = region == s.mreg[m][0] ? s.mreg[m][1] : s.mreg[m][0];
    f.kd = s.mkd[m];
    f.rho = s.mrho[m];
  }
  return f;
}

// Index of the hit primitive as the scene description numbers it (hash words).
__device__ __forceinline__ int hit_id(const SceneLDS& s, const Hit& h) {
  return h.kind == kHitMesh ? s.tri_orig[h.index] : h.index;
}

// Interface coefficients for direction d across normal n (any orientation),
// from medium (c1, Z1) into (c2, Z2): n_r faces the incident side; Snell from
// the sound-speed ratio; pressure coefficients from the impedances.
struct Coef { d3 nr; double ci, ct, Ar, At, RE; bool tir; };

__device__ __forceinline__ Coef coefficients(d3 d, d3 n, double c1, double Z1, double c2, double Z2) {
  Coef f;
  const double dn = dot(n, d);
  f.nr = dn > 0.0 ? d3{-n.x, -n.y, -n.z} : n;
  f.ci = dn > 0.0 ? dn : -dn;
  const double eta = c2 / c1;
  const double s2 = eta * eta * (1.0 - f.ci * f.ci);
  if (s2 >= 1.0) {
    f.tir = true; f.ct = 0.0; f.Ar = 1.0; f.At = 0.0; f.RE = 1.0;
    return f;
  }
  f.tir = false;
  f.ct = sqrt(1.0 - s2);
  const double zi = Z2 * f.ci, zt = Z1 * f.ct;
  const double inv = 1.0 / (zi + zt);
  f.Ar = (zi - zt) * inv;
  f.At = 2.0 * zi * inv;
  f.RE = f.Ar * f.Ar;
  return f;
}

// Orthonormal frame (b1, b2, n) about a unit normal n, branch-free form of
// Duff et al. (JCGT 2017); directions l = (lx, ly, lz) in it map to
// lx b1 + ly b2 + lz n.
struct Frame { d3 b1, b2; };
__device__ __forceinline__ Frame frame_of(d3 n) {
  const double sg = n.z >= 0.0 ? 1.0 : -1.0;
  const double aa = -1.0 / (sg + n.z);
  const double bb = n.x * n.y * aa;
  return Frame{d3{1.0 + sg * n.x * n.x * aa, sg * bb, -sg * n.x}, d3{bb, sg + n.y * n.y * aa, -n.y}};
}

// Transposed Jacobian of lx b1(n) + ly b2(n) + lz n with respect to n,
// applied to v (the frame depends on n through b1, b2).
__device__ __forceinline__ d3 frame_vjp(d3 n, double lx, double ly, double lz, d3 v) {
  const double sg = n.z >= 0.0 ? 1.0 : -1.0;
  const double aa = -1.0 / (sg + n.z);
  const double a2 = aa * aa;
  const double j_xx = lx * 2.0 * sg * n.x * aa + ly * n.y * aa + lz;
  const double j_xy = ly * n.x * aa;
  const double j_xz = lx * sg * n.x * n.x * a2 + ly * n.x * n.y * a2;
  const double j_yx = lx * sg * n.y * aa;
  const double j_yy = lx * sg * n.x * aa + ly * 2.0 * n.y * aa + lz;
  const double j_yz = lx * sg * n.x * n.y * a2 + ly * n.y * n.y * a2;
  const double j_zx = -lx * sg, j_zy = -ly, j_zz = lz;
  return d3{v.x * j_xx + v.y * j_yx + v.z * j_zx, v.x * j_xy + v.y * j_yy + v.z * j_zy,
            v.x * j_xz + v.y * j_yz + v.z * j_zz};
}

// Smith masking of one direction for GGX roughness rho at cosine c > 0.
__device__ __forceinline__ double smith_g1(double c, double rho) {
  return 2.0 * c / (c + sqrt(rho * rho + (1.0 - rho * rho) * c * c));
}

// Rough specular reflection (Eq. GGX_PDF): the specular share is mirrored
// about a microfacet normal m drawn with density D(m) (n.m) (tan theta_m =
// rho sqrt(u1 / (1 - u1)), azimuth 2 pi u2 in the frame about n_r); the
// weight takes the microfacet estimator factor
//   g = G1(n.i) G1(n.o) |i.m| / ((n.i) (n.m)),
// i = -d. A facet turned away from i, or an o below the surface, ends the
// path (ok = false). rho = 0 gives m = n_r.
struct Glossy { d3 dir; double g; bool ok; };
__device__ __forceinline__ Glossy glossy_reflect(d3 d, const Coef& f, double rho, double u1, double u2) {
  const Frame fr = frame_of(f.nr);
  const double th = rho * sqrt(u1 / (1.0 - u1));
  const double ch = 1.0 / sqrt(1.0 + th * th);
  const double sh = th * ch;
  const double phi = 2.0 * kPi * u2;
  const SinCos sc = sincos_ool(phi);
  const d3 m = fr.b1 * (sh * sc.c) + fr.b2 * (sh * sc.s) + f.nr * ch;
  Glossy o;
  const double wh = dot(d, m);
  o.dir = d - m * (2.0 * wh);
  const double co = dot(f.nr, o.dir);
  o.ok = wh < 0.0 && co > 0.0;
  o.g = o.ok ? smith_g1(f.ci, rho) * smith_g1(co, rho) * (-wh) / (f.ci * ch) : 0.0;
  return o;
}

// Entry j of a crossing list (selects, so the list stays in registers).
__device__ __forceinline__ void seg_get(const SegHits& L, int j, double* s, int* h) {
  double sv = L.s[0];
  int hv = L.h[0];
#pragma unroll
  for (int i = 1; i < kSegHits; ++i)
    if (j == i) { sv = L.s[i]; hv = L.h[i]; }
  *s = sv;
  *h = hv;
}

// Straight march of a receiver segment from x along the unit direction w to
// the point at distance r, starting in region reg: every crossed interface
// in order (pressure transmission coefficient each, blocked on total
// internal reflection), the travel time and the attenuation exponent summed
// over the legs. on_cross(j, s_j, hit word, surface, coefficients) sees
// crossing j (from 0) at distance s_j from x before its transmission is
// applied. A segment with max_legs(s) crossings or more is blocked.
struct March {
  double tof;     // tof0 + sum over legs of length / c
  double att;     // sum over legs of a * length
  double trans;   // product of the transmission coefficients
  int crossings;
  bool reached;
};

template <bool kMeshes, class OnCross>
__device__ __forceinline__ March receiver_march(const SceneLDS& S, d3 x, d3 w, double r, int reg,
                                                double tof0, int* stk, OnCross on_cross) {
  March m{tof0, 0.0, 1.0, 0, false};
  const int legs = max_legs(S);
  double lo = 0.0;   // distance of the last crossing taken
  for (;;) {
    const SegHits L = segment_hits<kMeshes>(S, x, w, lo, r, stk);
    for (int j = 0; j < L.n; ++j) {
      double sj;
      int hw;
      seg_get(L, j, &sj, &hw);
      if (!(sj > lo + kTMin)) continue;   // the surface point just crossed (a shared edge)
      const double ell = sj - lo;
      m.tof += ell * S.ic[reg];
      m.att += S.a[reg] * ell;
      lo = sj;
      const Hit h{hw >> 28, hw & 0x0FFFFFFF, sj};
      const d3 p = x + w * sj;
      const Surface sf = surface_of(S, h, p, reg);
      const Coef g = coefficients(w, sf.n, S.c[reg], S.Z[reg], S.c[sf.other], S.Z[sf.other]);
      on_cross(m.crossings, sj, hw, sf, g);
      ++m.crossings;
      if (g.tir) return m;
      m.trans *= g.At;
      reg = sf.other;
      if (m.crossings >= legs) return m;
    }
    if (L.n < kSegHits) break;   // every crossing up to r was in the list
  }
  const double ell = r - lo;
  m.tof += ell * S.ic[reg];
  m.att += S.a[reg] * ell;
  m.reached = true;
  return m;
}

__device__ __forceinline__ double elem_x(const ProbeView& p, int e) {
  return ((double)e - 0.5 * (double)(p.n_elem - 1)) * p.pitch;
}


}  // namespace usrt
