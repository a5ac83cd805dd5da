// Device geometry and interface physics shared by the forward transport and
// the replay backward, so that both take identical discrete decisions.
#pragma once

#include "common.h"

namespace usrt {

struct Hit { int kind; int index; double t; };

__device__ __forceinline__ d3 vtx(const double* v, int i) {
  return d3{v[3 * i], v[3 * i + 1], v[3 * i + 2]};
}
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
  return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Ray against one fp32 child box padded by kPad (absorbs the rounding of the
// ray to fp32); entry distance in *t0, culled beyond lim.
__device__ __forceinline__ bool slab(const float* lo, const float* hi, float ox, float oy, float oz,
                                     float ix, float iy, float iz, float lim, float* t0) {
  constexpr float kPad = 1e-6f;
  const float ax = (lo[0] - kPad - ox) * ix, bx = (hi[0] + kPad - ox) * ix;
  const float ay = (lo[1] - kPad - oy) * iy, by = (hi[1] + kPad - oy) * iy;
  const float az = (lo[2] - kPad - oz) * iz, bz = (hi[2] + kPad - oz) * iz;
  const float tmin = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
  const float tmax = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
  *t0 = tmin;
  return tmin <= tmax && tmin <= lim;
}

// Moller-Trumbore in fp64 on a leaf-order triangle record, edges included;
// distance or -1.
__device__ __forceinline__ double rec_distance(const TriRec& r, d3 o, d3 d) {
  const d3 e1{r.e1[0], r.e1[1], r.e1[2]}, e2{r.e2[0], r.e2[1], r.e2[2]};
  const d3 pv = cross(d, e2);
  const double det = dot(e1, pv);
  if (det == 0.0) return -1.0;
  const double inv = 1.0 / det;
  const d3 sv = o - d3{r.p0[0], r.p0[1], r.p0[2]};
  const double u = dot(sv, pv) * inv;
  if (u < 0.0 || u > 1.0) return -1.0;
  const d3 qv = cross(sv, e1);
  const double v = dot(d, qv) * inv;
  if (v < 0.0 || u + v > 1.0) return -1.0;
  return dot(e2, qv) * inv;
}

// Closest triangle in (kTMin, best) by walking the hierarchy near child
// first. One step handles one inner node (both child boxes tested against the
// ray in fp32; the farther of two hit children is pushed) or one leaf (its
// triangles intersected in fp64). The stack lives in LDS, interleaved across
// the block's threads (entry i of this thread at stk[i * blockDim.x]); it
// holds at most one entry per inner level.
__device__ __forceinline__ void mesh_closest(const SceneLDS& s, d3 o, d3 d, double& best, int& best_tri,
                                             int* stk) {
  constexpr float kPad = 1e-6f;
  const float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
  const float ix = fabs(d.x) > 1e-30 ? (float)(1.0 / d.x) : copysignf(1e30f, (float)d.x);
  const float iy = fabs(d.y) > 1e-30 ? (float)(1.0 / d.y) : copysignf(1e30f, (float)d.y);
  const float iz = fabs(d.z) > 1e-30 ? (float)(1.0 / d.z) : copysignf(1e30f, (float)d.z);
  const int step = blockDim.x;
  int sp = 0, cur = 0;
  for (;;) {
    if (cur >= 0) {
      const BvhNode n = s.nodes[cur];
      const float lim = (float)best * 1.0001f + kPad;
      float tl, tr;
      const bool hl = slab(n.lo_l, n.hi_l, ox, oy, oz, ix, iy, iz, lim, &tl);
      const bool hr = slab(n.lo_r, n.hi_r, ox, oy, oz, ix, iy, iz, lim, &tr);
      if (hl && hr) {
        const bool left_first = tl <= tr;
        // the build bounds the inner depth by stack_cap, so the push always fits
        if (sp < s.stack_cap) { stk[sp * step] = left_first ? n.right : n.left; ++sp; }
        cur = left_first ? n.left : n.right;
        continue;
      }
      if (hl) { cur = n.left; continue; }
      if (hr) { cur = n.right; continue; }
    } else {
      const int first = (~cur) >> 4, cnt = (~cur) & 15;
      for (int i = first; i < first + cnt; ++i) {
        const double t = rec_distance(s.trec[i], o, d);
        if (t > kTMin && t < best) { best = t; best_tri = i; }
      }
    }
    if (sp == 0) break;
    --sp;
    cur = stk[sp * step];
  }
}

// Closest surface along o + t d with kTMin < t < tmax among the planes, the
// spheres, the meshes and, when `with_array` and the ray moves up, the array
// face z = 0.
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
  if (s.n_meshes > 0) {
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
  return s.n_planes + 2 * s.n_spheres + kMeshLegs * s.n_meshes + 1;
}

// Unit face normal of leaf-order triangle i, from the current geometry.
__device__ __forceinline__ d3 tri_normal(const SceneLDS& s, int i) {
  const TriRec& r = s.trec[i];
  const d3 nu = cross(d3{r.e1[0], r.e1[1], r.e1[2]}, d3{r.e2[0], r.e2[1], r.e2[2]});
  return nu * (1.0 / sqrt(dot(nu, nu)));
}

struct Surface { d3 n; int other; double kd; };

__device__ __forceinline__ Surface surface_of(const SceneLDS& s, const Hit& h, d3 x, int region) {
  Surface f;
  if (h.kind == kHitPlane) {
    f.n = d3{0.0, 0.0, 1.0};
    f.other = region == s.pr[h.index][0] ? s.pr[h.index][1] : s.pr[h.index][0];
    f.kd = s.pkd[h.index];
  } else if (h.kind == kHitSphere) {
    const double ir = 1.0 / s.sr[h.index];
    f.n = d3{(x.x - s.sx[h.index]) * ir, (x.y - s.sy[h.index]) * ir, (x.z - s.sz[h.index]) * ir};
    f.other = region == s.sreg[h.index][0] ? s.sreg[h.index][1] : s.sreg[h.index][0];
    f.kd = s.skd[h.index];
  } else {
    const int m = s.tri[h.index].w;
    f.n = tri_normal(s, h.index);
    f.other = region == s.mreg[m][0] ? s.mreg[m][1] : s.mreg[m][0];
    f.kd = s.mkd[m];
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

__device__ __forceinline__ double elem_x(const ProbeView& p, int e) {
  return ((double)e - 0.5 * (double)(p.n_elem - 1)) * p.pitch;
}


}  // namespace usrt
