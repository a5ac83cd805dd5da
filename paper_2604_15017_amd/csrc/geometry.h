// Device geometry and interface physics shared by the forward transport and
// the replay backward, so that both take identical discrete decisions.
#pragma once

#include "common.h"

namespace usrt {

struct Hit { int kind; int index; double t; };

// Closest surface along o + t d with t > kTMin among the planes, the spheres
// and, when `with_array` and the ray moves up, the array face z = 0.
__device__ __forceinline__ Hit closest_hit(const SceneLDS& s, d3 o, d3 d, bool with_array) {
  Hit h{kHitNone, -1, 0.0};
  double best = INFINITY;
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
  return h;
}

struct Surface { d3 n; int other; double kd; };

__device__ __forceinline__ Surface surface_of(const SceneLDS& s, const Hit& h, d3 x, int region) {
  Surface f;
  if (h.kind == kHitPlane) {
    f.n = d3{0.0, 0.0, 1.0};
    f.other = region == s.pr[h.index][0] ? s.pr[h.index][1] : s.pr[h.index][0];
    f.kd = s.pkd[h.index];
  } else {
    const double ir = 1.0 / s.sr[h.index];
    f.n = d3{(x.x - s.sx[h.index]) * ir, (x.y - s.sy[h.index]) * ir, (x.z - s.sz[h.index]) * ir};
    f.other = region == s.sreg[h.index][0] ? s.sreg[h.index][1] : s.sreg[h.index][0];
    f.kd = s.skd[h.index];
  }
  return f;
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

__device__ __forceinline__ void splat(float* h, long row, int n_t, double fs, double t, double a) {
  const double x = t * fs;
  if (!(x > -1.0 && x < (double)n_t)) return;   // also rejects NaN
  const double j0d = floor(x);
  const double f = x - j0d;
  const int j0 = (int)j0d;
  float* r = h + row * (long)n_t;
  if (j0 >= 0) unsafeAtomicAdd(r + j0, (float)(a * (1.0 - f)));
  if (j0 + 1 < n_t) unsafeAtomicAdd(r + j0 + 1, (float)(a * f));
}

__device__ __forceinline__ double elem_x(const ProbeView& p, int e) {
  return ((double)e - 0.5 * (double)(p.n_elem - 1)) * p.pitch;
}


}  // namespace usrt
