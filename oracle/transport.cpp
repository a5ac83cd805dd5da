// FP64 reference transport for full-path Monte-Carlo ultrasound ray tracing.
//
// TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU path is
// checked against. Only tests, the smoke check and the CPU-baseline leg of the
// benchmark may load it. It shares no code with the GPU library.
//
// What it computes (paper Sec. 2.3, "Algorithmic Implementation of the
// Ray-Tracing Model"), step by step and in the paper's order, in FP64:
//   emission    (Sec. 2.3.1, Eq. directivity)  origin on the element face,
//               steering direction, transmit delay as a time stamp, weight
//               f_d / N;
//   traversal   (Sec. 2.3.2) closest hit; specular reflection; Snell
//               refraction; pressure Fresnel coefficients with the energy
//               split A_r^2 used as the branch probability; a Lambertian
//               lobe stands in for the rough (GGX) part; attenuation along
//               each segment; bounce cap;
//   transducer sampling (Sec. 2.3.3, Eq. cutoff): a receiver-directed
//               secondary ray to the centre of a uniformly chosen element
//               after each interaction with a diffuse-capable surface, with
//               the element-pick probability in the weight, and the
//               receive directivity;
//   deposit     (Sec. 2.3.4) each contribution is splatted at its time of
//               flight into h[tx][element][sample] with a linear tent.
// Gradients (Sec. 3.2, Eq. chain_rule): derivatives of the fixed-sample
// estimator with respect to the scene parameters, with every discrete choice
// frozen, computed here by forward-mode dual numbers and contracted with a
// given dL/dh.
//
// The readings taken where the paper is silent are listed in the design
// notes of the repository; each is marked "reading" below.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// --------------------------------------------------------------------------
// Forward-mode dual number with up to MAXD tangent directions.
// --------------------------------------------------------------------------
constexpr int MAXD = 64;
thread_local int g_nd = 0;   // number of active tangent directions

struct Dual {
  double v;
  double d[MAXD];
  Dual() : v(0) { for (int i = 0; i < g_nd; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < g_nd; ++i) d[i] = 0; }
};

inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < g_nd; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < g_nd; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual sqrt(const Dual& a) {
  Dual r(std::sqrt(a.v));
  for (int i = 0; i < g_nd; ++i) r.d[i] = r.v > 0 ? a.d[i] / (2 * r.v) : 0.0;
  return r;
}
inline Dual exp(const Dual& a) { Dual r(std::exp(a.v)); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * r.v; return r; }
inline Dual acos(const Dual& a) {
  Dual r(std::acos(a.v));
  double s = 1.0 - a.v * a.v;
  for (int i = 0; i < g_nd; ++i) r.d[i] = s > 0 ? -a.d[i] / std::sqrt(s) : 0.0;
  return r;
}
inline Dual sin(const Dual& a) { Dual r(std::sin(a.v)); double c = std::cos(a.v); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * c; return r; }
inline Dual cos(const Dual& a) { Dual r(std::cos(a.v)); double s = -std::sin(a.v); for (int i = 0; i < g_nd; ++i) r.d[i] = a.d[i] * s; return r; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::sqrt; using std::exp; using std::acos; using std::sin; using std::cos;

template <class T> struct V3 { T x, y, z; };
template <class T> inline V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> inline V3<T> operator*(const V3<T>& a, const T& s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> inline T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// --------------------------------------------------------------------------
// Counter-based generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror,
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from
// its published definition. key = (seed, 0); counter = (ray id, transmit id,
// event index, 0); event 0 is emission, event k >= 1 is the k-th interaction.
// --------------------------------------------------------------------------
void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform in (0,1) with 23 random bits, odd multiples of 2^-24: exact in
// both float and double (reading: so that float and double comparisons
// against it agree).
inline double uniform_from(uint64_t x) { return ((double)(x >> 41) + 0.5) * (1.0 / 8388608.0); }

struct U4 { double u[4]; };
U4 draw(uint64_t seed, uint64_t ray_id, uint32_t tx_id, uint32_t event) {
  uint64_t ctr[4] = {ray_id, (uint64_t)tx_id, (uint64_t)event, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t o[4];
  philox4x64_10(ctr, key, o);
  return U4{{uniform_from(o[0]), uniform_from(o[1]), uniform_from(o[2]), uniform_from(o[3])}};
}

// Per-ray decision hash used to count paths whose discrete choices differ
// between two implementations: the sum (mod 2^64) over the path's events of
// mix(tag, event index, word), mix being the SplitMix64 finaliser. A sum does
// not depend on the order in which events are visited.
struct PathHash {
  uint64_t h = 0;
  void add(uint32_t tag, uint32_t k, uint32_t word) {
    uint64_t z = ((uint64_t)tag << 60) | ((uint64_t)(k & 0xFFFu) << 48) | (uint64_t)word;
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    h += z ^ (z >> 31);
  }
};
// event tags
enum { EV_HIT = 1, EV_ARRAY = 2, EV_BRANCH = 3, EV_NEE = 4 };

}  // namespace

extern "C" {

// Plain-C descriptions filled from Python (oracle/__init__.py mirrors them).
struct OrSceneDesc {
  int n_regions, n_planes, n_spheres;
  const int32_t* plane_regions;   // [n_planes][2]: above, below
  const double* plane_kd;         // [n_planes]
  const int32_t* sphere_regions;  // [n_spheres][2]: inside, outside
  const double* sphere_kd;        // [n_spheres]
  int start_region;
  // closed triangle meshes; vertex v moves as vrest + sum_j q_j basis[v][j] vnormal[v]
  int n_meshes, n_basis;
  const int32_t* mesh_regions;    // [n_meshes][2]: inside, outside
  const double* mesh_kd;          // [n_meshes]
  int64_t n_vertices, n_triangles;
  const double* vrest;            // [V][3]
  const double* vnormal;          // [V][3]
  const double* vbasis;           // [V][n_basis]
  const int32_t* vmesh;           // [V]
  const int32_t* tris;            // [T][3]
  const int32_t* tmesh;           // [T]
  int mesh_bruteforce;            // test hook: 1 = test every triangle instead of the BVH
  // cylinders along y: (x - cx)^2 + (z - cz)^2 = R^2 for every y
  int n_cylinders;
  const int32_t* cylinder_regions;  // [n_cylinders][2]: inside, outside
  const double* cylinder_kd;        // [n_cylinders]
};

struct OrProbeDesc {
  int n_elem;
  double pitch, elem_width, elem_height, f0, n_cycles, fs;
  int n_t;
  double c_ref, alpha_main, alpha_cut;
};

struct OrRunDesc {
  int n_tx;
  const double* angles;      // [n_tx]
  const uint32_t* tx_ids;    // [n_tx]
  uint64_t seed;
  int rays_per_elem;
  int64_t ray_begin, ray_count;   // per transmit, ray id range
  int max_bounces;
  int nee_mode;              // 0: receiver-directed secondary rays (default);
                             // 1: none; paths after a diffuse bounce count when they hit an element
  int n_threads;             // 0 = OpenMP default
  // Selection probabilities (test hook for finite differences of the
  // estimator with its sampling density held fixed): 0 = computed; 1 =
  // computed and recorded into prob_buf; 2 = read from prob_buf. prob_buf is
  // [n_tx][ray_count][max_bounces], the reflected-energy fraction R_E used at
  // interaction k = 1..max_bounces.
  int prob_mode;
  double* prob_buf;
};

struct OrContrib { int32_t tx, elem; double t, a; int64_t ray; };

}  // extern "C"

namespace {

constexpr double TMIN = 1e-6;   // reading: self-intersection guard of 1 um
constexpr double PI = 3.14159265358979323846;

enum HitKind { HIT_NONE = 0, HIT_PLANE = 1, HIT_SPHERE = 2, HIT_ARRAY = 3, HIT_MESH = 4, HIT_CYLINDER = 5 };

// Bounding-volume hierarchy over the mesh triangles (median split along the
// longest axis of the centroids, at most 4 triangles per leaf). It only
// accelerates the closest-hit search; the hit is the same as a linear scan.
struct BNode { double lo[3], hi[3]; int left, right, first, count; };

struct Bvh {
  std::vector<BNode> nodes;
  std::vector<int> order;   // triangle ids in leaf order
  void build(const std::vector<double>& vp, const int32_t* tris, int64_t n_tri) {
    order.resize(n_tri);
    for (int64_t i = 0; i < n_tri; ++i) order[i] = (int)i;
    std::vector<double> cen(3 * n_tri);
    for (int64_t i = 0; i < n_tri; ++i)
      for (int k = 0; k < 3; ++k)
        cen[3 * i + k] = (vp[3 * tris[3 * i] + k] + vp[3 * tris[3 * i + 1] + k] + vp[3 * tris[3 * i + 2] + k]) / 3.0;
    nodes.clear();
    if (n_tri) split(vp, tris, cen, 0, (int)n_tri);
  }
  int split(const std::vector<double>& vp, const int32_t* tris, const std::vector<double>& cen,
            int first, int count) {
    int id = (int)nodes.size();
    nodes.push_back(BNode{});
    BNode nd;
    for (int k = 0; k < 3; ++k) { nd.lo[k] = INFINITY; nd.hi[k] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = first; i < first + count; ++i) {
      int t = order[i];
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
          double x = vp[3 * tris[3 * t + j] + k];
          nd.lo[k] = std::min(nd.lo[k], x); nd.hi[k] = std::max(nd.hi[k], x);
        }
      for (int k = 0; k < 3; ++k) { clo[k] = std::min(clo[k], cen[3 * t + k]); chi[k] = std::max(chi[k], cen[3 * t + k]); }
    }
    if (count <= 4) {
      nd.left = nd.right = -1; nd.first = first; nd.count = count;
      nodes[id] = nd;
      return id;
    }
    int ax = 0;
    for (int k = 1; k < 3; ++k) if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    int mid = first + count / 2;
    std::nth_element(order.begin() + first, order.begin() + mid, order.begin() + first + count,
                     [&](int a, int b) { return cen[3 * a + ax] < cen[3 * b + ax]; });
    nd.first = first; nd.count = 0;
    nd.left = split(vp, tris, cen, first, mid - first);
    nd.right = split(vp, tris, cen, mid, first + count - mid);
    nodes[id] = nd;
    return id;
  }
};

template <class T>
struct Model {
  const OrSceneDesc* sd;
  const OrProbeDesc* pd;
  const OrRunDesc* rd;
  std::vector<T> c, Z, a;               // per region: speed, impedance, amplitude attenuation [Np/m]
  std::vector<T> pz;                    // plane depths
  std::vector<V3<T>> sc; std::vector<T> sr;  // sphere centres, radii
  std::vector<T> ccx, ccz, cr;          // cylinder axes (x, z) and radii
  std::vector<T> rho_p, rho_s, rho_c, rho_m;   // GGX roughness of planes, spheres, cylinders, meshes
  std::vector<T> q;                     // mesh displacement coefficients [n_meshes][n_basis]
  std::vector<double> vpos;             // current vertex positions (values) [V][3]
  Bvh bvh;
};

// Current position of mesh vertex v as a function of the displacement coefficients.
template <class T>
V3<T> vertex(const Model<T>& m, int v) {
  const OrSceneDesc* sd = m.sd;
  const int mesh = sd->vmesh[v];
  T s(0.0);
  for (int j = 0; j < sd->n_basis; ++j) s = s + m.q[mesh * sd->n_basis + j] * sd->vbasis[(int64_t)v * sd->n_basis + j];
  return V3<T>{sd->vrest[3 * v] + s * sd->vnormal[3 * v], sd->vrest[3 * v + 1] + s * sd->vnormal[3 * v + 1],
               sd->vrest[3 * v + 2] + s * sd->vnormal[3 * v + 2]};
}

// Moller-Trumbore on values, edges included; returns the distance or -1.
double tri_hit_value(const Model<double>* dummy, const std::vector<double>& vp, const int32_t* tri,
                     const double* o, const double* d) {
  (void)dummy;
  const double* p0 = &vp[3 * tri[0]];
  const double* p1 = &vp[3 * tri[1]];
  const double* p2 = &vp[3 * tri[2]];
  double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
  double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
  if (det == 0.0) return -1.0;
  double inv = 1.0 / det;
  double sv[3] = {o[0] - p0[0], o[1] - p0[1], o[2] - p0[2]};
  double u = (sv[0] * pv[0] + sv[1] * pv[1] + sv[2] * pv[2]) * inv;
  if (u < 0.0 || u > 1.0) return -1.0;
  double qv[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2], sv[0] * e1[1] - sv[1] * e1[0]};
  double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
  if (v < 0.0 || u + v > 1.0) return -1.0;
  return (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
}

// Closest triangle with distance in (TMIN, best): linear scan or BVH walk.
template <class T>
void mesh_closest(const Model<T>& m, const double* o, const double* d, double* best, int* best_tri) {
  const OrSceneDesc* sd = m.sd;
  if (sd->mesh_bruteforce) {
    for (int64_t t = 0; t < sd->n_triangles; ++t) {
      double tt = tri_hit_value(nullptr, m.vpos, sd->tris + 3 * t, o, d);
      if (tt > TMIN && tt < *best) { *best = tt; *best_tri = (int)t; }
    }
    return;
  }
  if (m.bvh.nodes.empty()) return;
  std::vector<int> stack;
  stack.push_back(0);
  while (!stack.empty()) {
    const BNode& nd = m.bvh.nodes[stack.back()];
    stack.pop_back();
    // slab test of the node box
    double t0 = 0.0, t1 = *best;
    bool hit = true;
    for (int k = 0; k < 3 && hit; ++k) {
      if (d[k] == 0.0) {
        if (o[k] < nd.lo[k] || o[k] > nd.hi[k]) hit = false;
        continue;
      }
      double ta = (nd.lo[k] - o[k]) / d[k], tb = (nd.hi[k] - o[k]) / d[k];
      if (ta > tb) std::swap(ta, tb);
      t0 = std::max(t0, ta); t1 = std::min(t1, tb);
      if (t0 > t1) hit = false;
    }
    if (!hit) continue;
    if (nd.left < 0) {
      for (int i = nd.first; i < nd.first + nd.count; ++i) {
        int t = m.bvh.order[i];
        double tt = tri_hit_value(nullptr, m.vpos, sd->tris + 3 * t, o, d);
        if (tt > TMIN && tt < *best) { *best = tt; *best_tri = t; }
      }
    } else {
      stack.push_back(nd.left);
      stack.push_back(nd.right);
    }
  }
}

// Distance to the plane of triangle t along (o, w), and its unit normal, as
// functions of the displacement coefficients.
template <class T>
void tri_geometry(const Model<T>& m, int t, const V3<T>& o, const V3<T>& w, T* dist, V3<T>* n) {
  const int32_t* tr = m.sd->tris + 3 * t;
  V3<T> p0 = vertex(m, tr[0]), p1 = vertex(m, tr[1]), p2 = vertex(m, tr[2]);
  V3<T> e1 = p1 - p0, e2 = p2 - p0;
  V3<T> nu{e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
  if (dist) *dist = dot(nu, p0 - o) / dot(nu, w);
  if (n) {
    T len = sqrt(dot(nu, nu));
    *n = nu * (1.0 / len);
  }
}

template <class T>
struct Hit { int kind; int index; T t; };

// Closest surface along o + t w with t > TMIN; the array face z = 0 is a
// candidate only when `with_array` and the ray moves toward it.
template <class T>
Hit<T> closest_hit(const Model<T>& m, const V3<T>& o, const V3<T>& w, bool with_array) {
  Hit<T> best{HIT_NONE, -1, T(0.0)};
  double best_t = INFINITY;
  if (val(w.z) != 0.0) {
    for (int k = 0; k < m.sd->n_planes; ++k) {
      T t = (m.pz[k] - o.z) / w.z;
      if (val(t) > TMIN && val(t) < best_t) { best = {HIT_PLANE, k, t}; best_t = val(t); }
    }
  }
  for (int k = 0; k < m.sd->n_spheres; ++k) {
    V3<T> oc = o - m.sc[k];
    T b = dot(oc, w);
    T cc = dot(oc, oc) - m.sr[k] * m.sr[k];
    T disc = b * b - cc;
    if (val(disc) < 0) continue;
    T sq = sqrt(disc);
    T t1 = -b - sq, t2 = -b + sq;
    T t = val(t1) > TMIN ? t1 : t2;
    if (val(t) > TMIN && val(t) < best_t) { best = {HIT_SPHERE, k, t}; best_t = val(t); }
  }
  // cylinder: |(o + t w - c) projected on the x-z plane| = R, a t^2 + 2 b t + cc = 0
  for (int k = 0; k < m.sd->n_cylinders; ++k) {
    T ox = o.x - m.ccx[k], oz = o.z - m.ccz[k];
    T a = w.x * w.x + w.z * w.z;
    if (val(a) <= 0.0) continue;            // parallel to the axis
    T b = ox * w.x + oz * w.z;
    T cc = ox * ox + oz * oz - m.cr[k] * m.cr[k];
    T disc = b * b - a * cc;
    if (val(disc) < 0) continue;
    T sq = sqrt(disc);
    T t1 = (-b - sq) / a, t2 = (-b + sq) / a;
    T t = val(t1) > TMIN ? t1 : t2;
    if (val(t) > TMIN && val(t) < best_t) { best = {HIT_CYLINDER, k, t}; best_t = val(t); }
  }
  if (m.sd->n_meshes > 0) {
    double ov[3] = {val(o.x), val(o.y), val(o.z)}, wv[3] = {val(w.x), val(w.y), val(w.z)};
    double bt = best_t;
    int tri = -1;
    mesh_closest(m, ov, wv, &bt, &tri);
    if (tri >= 0) {
      T t;
      tri_geometry(m, tri, o, w, &t, (V3<T>*)nullptr);
      best = {HIT_MESH, tri, t};
      best_t = bt;
    }
  }
  if (with_array && val(w.z) < 0.0) {
    T t = -o.z / w.z;
    if (val(t) > TMIN && val(t) < best_t) { best = {HIT_ARRAY, -1, t}; best_t = val(t); }
  }
  return best;
}

// Geometric normal of the surface that was hit, and the region across it.
template <class T>
void surface_at(const Model<T>& m, const Hit<T>& h, const V3<T>& x, int region,
                V3<T>* n, int* other, double* kd, T* rho = nullptr) {
  if (h.kind == HIT_PLANE) {
    *n = {T(0.0), T(0.0), T(1.0)};
    const int32_t* pr = m.sd->plane_regions + 2 * h.index;
    *other = region == pr[0] ? pr[1] : pr[0];
    *kd = m.sd->plane_kd[h.index];
    if (rho) *rho = m.rho_p[h.index];
  } else if (h.kind == HIT_SPHERE) {
    T inv_r = 1.0 / m.sr[h.index];
    *n = (x - m.sc[h.index]) * inv_r;
    const int32_t* sr = m.sd->sphere_regions + 2 * h.index;
    *other = region == sr[0] ? sr[1] : sr[0];
    *kd = m.sd->sphere_kd[h.index];
    if (rho) *rho = m.rho_s[h.index];
  } else if (h.kind == HIT_CYLINDER) {
    T inv_r = 1.0 / m.cr[h.index];
    *n = {(x.x - m.ccx[h.index]) * inv_r, T(0.0), (x.z - m.ccz[h.index]) * inv_r};
    const int32_t* cr = m.sd->cylinder_regions + 2 * h.index;
    *other = region == cr[0] ? cr[1] : cr[0];
    *kd = m.sd->cylinder_kd[h.index];
    if (rho) *rho = m.rho_c[h.index];
  } else {   // mesh triangle: flat face normal
    V3<T> zero{T(0.0), T(0.0), T(1.0)};
    tri_geometry(m, h.index, x, zero, (T*)nullptr, n);
    const int mesh = m.sd->tmesh[h.index];
    const int32_t* mr = m.sd->mesh_regions + 2 * mesh;
    *other = region == mr[0] ? mr[1] : mr[0];
    *kd = m.sd->mesh_kd[mesh];
    if (rho) *rho = m.rho_m[mesh];
  }
}

// Interface between incident medium 1 and medium 2 for direction w and
// normal n (Sec. 2.3.2). n_r is n turned toward the incident side. Direction
// of the transmitted ray from the sound-speed ratio (Snell); coefficients
// from the impedances. Reading of the printed coefficient: the standard
// fluid-fluid pressure coefficients
//   A_r = (Z2 cos_i - Z1 cos_t) / (Z2 cos_i + Z1 cos_t),
//   A_t = 2 Z2 cos_i / (Z2 cos_i + Z1 cos_t),
// which reduce to (Z2 - Z1)/(Z2 + Z1) at normal incidence; A_r^2 is the
// reflected energy fraction that sets the branch probability.
template <class T>
struct Interface { V3<T> n_r; T cos_i, cos_t, Ar, At; double RE; bool tir; };

template <class T>
Interface<T> interface_at(const V3<T>& w, const V3<T>& n, const T& c1, const T& Z1,
                          const T& c2, const T& Z2) {
  Interface<T> f;
  bool flip = val(dot(n, w)) > 0.0;
  f.n_r = flip ? V3<T>{-n.x, -n.y, -n.z} : n;
  f.cos_i = -dot(f.n_r, w);
  T eta = c2 / c1;
  T sin2_t = eta * eta * (1.0 - f.cos_i * f.cos_i);
  if (val(sin2_t) >= 1.0) {
    f.tir = true;
    f.cos_t = T(0.0); f.Ar = T(1.0); f.At = T(0.0); f.RE = 1.0;
    return f;
  }
  f.tir = false;
  f.cos_t = sqrt(1.0 - sin2_t);
  T D = Z2 * f.cos_i + Z1 * f.cos_t;
  f.Ar = (Z2 * f.cos_i - Z1 * f.cos_t) / D;
  f.At = 2.0 * Z2 * f.cos_i / D;
  f.RE = val(f.Ar) * val(f.Ar);
  return f;
}

template <class T>
V3<T> reflect_dir(const V3<T>& w, const Interface<T>& f) {  // w + 2 (n.(-w)) n
  return w + f.n_r * (2.0 * f.cos_i);
}

template <class T>
V3<T> refract_dir(const V3<T>& w, const Interface<T>& f, const T& eta) {
  return w * eta + f.n_r * (eta * f.cos_i - f.cos_t);
}

// Cosine-weighted direction about n (Lambertian lobe), in the orthonormal
// frame of Duff et al., "Building an orthonormal basis, revisited" (JCGT 2017).
template <class T>
V3<T> cosine_dir(const V3<T>& n, double u1, double u2) {
  double sgn = val(n.z) >= 0.0 ? 1.0 : -1.0;
  T a = -1.0 / (sgn + n.z);
  T b = n.x * n.y * a;
  V3<T> b1{1.0 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x};
  V3<T> b2{b, sgn + n.y * n.y * a, -n.y};
  double phi = 2.0 * PI * u1, rr = std::sqrt(u2);
  double lx = rr * std::cos(phi), ly = rr * std::sin(phi), lz = std::sqrt(1.0 - u2);
  return b1 * T(lx) + b2 * T(ly) + n * T(lz);
}

// Rough specular reflection (Eq. GGX_PDF). Reading: the specular share of
// the reflection is mirrored about a microfacet normal h drawn with density
// D(h) (n.h) (GGX with roughness rho: tan^2 theta_h = rho^2 u1 / (1 - u1),
// azimuth 2 pi u2, in the same orthonormal frame about n_r as the
// Lambertian lobe); the path weight takes the microfacet estimator factor
//   G1(n.i) G1(n.o) |i.h| / ((n.i) (n.h)),
//   G1(c) = 2 c / (c + sqrt(rho^2 + (1 - rho^2) c^2))   (Smith, separable),
// i = -w the direction towards the source, o the reflected direction. The
// Fresnel amplitude and the reflect / refract / diffuse choice stay those of
// the macroscopic normal. A microfacet facing away from i, or an o below the
// surface, ends the path (factor 0). rho = 0 gives h = n_r and the mirror.
template <class T>
struct Glossy { V3<T> dir; T g; bool ok; };

template <class T>
T smith_g1(const T& c, const T& rho) {
  return 2.0 * c / (c + sqrt(rho * rho + (1.0 - rho * rho) * c * c));
}

template <class T>
Glossy<T> glossy_reflect(const V3<T>& w, const Interface<T>& f, const T& rho, double u1, double u2) {
  const V3<T>& n = f.n_r;
  double sgn = val(n.z) >= 0.0 ? 1.0 : -1.0;
  T a = -1.0 / (sgn + n.z);
  T b = n.x * n.y * a;
  V3<T> b1{1.0 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x};
  V3<T> b2{b, sgn + n.y * n.y * a, -n.y};
  T tan_h = rho * std::sqrt(u1 / (1.0 - u1));   // rho >= 0; smooth in rho at 0
  T cos_h = 1.0 / sqrt(1.0 + tan_h * tan_h);
  T sin_h = tan_h * cos_h;
  double phi = 2.0 * PI * u2;
  V3<T> h = b1 * (sin_h * std::cos(phi)) + b2 * (sin_h * std::sin(phi)) + n * cos_h;
  Glossy<T> out;
  T wh = dot(w, h);
  out.dir = w - h * (2.0 * wh);
  T cos_o = dot(n, out.dir);
  out.ok = val(wh) < 0.0 && val(cos_o) > 0.0;
  if (!out.ok) { out.g = T(0.0); return out; }
  out.g = smith_g1(f.cos_i, rho) * smith_g1(cos_o, rho) * (-wh) / (f.cos_i * cos_h);
  return out;
}

// Receive directivity (Eq. cutoff), angle alpha = acos(n . w_i).
template <class T>
T directivity(const OrProbeDesc* pd, const T& cos_a) {
  double c = std::min(1.0, std::max(-1.0, val(cos_a)));
  double al = std::acos(c);
  if (al <= pd->alpha_main) return T(1.0);
  if (al > pd->alpha_cut) return T(0.0);
  return (pd->alpha_cut - acos(cos_a)) / (pd->alpha_cut - pd->alpha_main);
}

template <class T> struct Sink;

template <>
struct Sink<double> {
  std::vector<OrContrib>* out;
  void deposit(int tx, int e, double t, double a, int64_t ray) { out->push_back({tx, e, t, a, ray}); }
};

template <>
struct Sink<Dual> {
  std::vector<OrContrib>* out;
  const double* g_h;      // [n_tx][n_elem][n_t]
  const OrProbeDesc* pd;
  double* g_acc;          // [g_nd]
  void deposit(int tx, int e, const Dual& t, const Dual& a, int64_t ray) {
    out->push_back({tx, e, t.v, a.v, ray});
    // tent splat h[j0] += a (1 - f), h[j0+1] += a f with f = t fs - j0
    double x = t.v * pd->fs;
    double j0d = std::floor(x);
    double f = x - j0d;
    long j0 = (long)j0d;
    const double* g = g_h + ((long)tx * pd->n_elem + e) * (long)pd->n_t;
    double g0 = (j0 >= 0 && j0 < pd->n_t) ? g[j0] : 0.0;
    double g1 = (j0 + 1 >= 0 && j0 + 1 < pd->n_t) ? g[j0 + 1] : 0.0;
    double ga = g0 * (1.0 - f) + g1 * f;
    double gt = a.v * pd->fs * (g1 - g0);
    for (int i = 0; i < g_nd; ++i) g_acc[i] += ga * a.d[i] + gt * t.d[i];
  }
};

// Receiver-directed secondary ray (Sec. 2.3.3) from x, where the path has
// weight w and time t, toward the centre of element e2. Reading: the
// secondary ray goes straight through the interfaces it crosses, taking the
// transmission coefficient of each (zero beyond the critical angle) and the
// attenuation and travel time of every medium on the way. Lambertian lobe
// kd * A_r * cos_o / pi, solid angle of the element A_el cos_el / r^2, and
// the factor N_e for the uniform element choice.
template <class T>
void receiver_ray(const Model<T>& m, Sink<T>& sink, PathHash& ph, int64_t* segs, int txi,
                  int64_t ray, int k, int region, const V3<T>& x, const Interface<T>& f, double kd,
                  const T& w, const T& t, int e2) {
  const OrProbeDesc* pd = m.pd;
  double xe = (e2 - 0.5 * (pd->n_elem - 1)) * pd->pitch;
  V3<T> y{T(xe), T(0.0), T(0.0)};
  V3<T> d = y - x;
  T r = sqrt(dot(d, d));
  V3<T> we = d * (1.0 / r);
  T cos_o = dot(f.n_r, we);
  // NEE event word: element | status << 16 | crossings << 20
  // (status 0 deposited, 1 element behind the surface, 2 outside the receive
  // cutoff, 3 blocked by total internal reflection)
  if (val(cos_o) <= 0.0) { ph.add(EV_NEE, k, (uint32_t)e2 | (1u << 16)); return; }
  T cos_el = -we.z;
  T fd = directivity(pd, cos_el);
  if (val(fd) == 0.0) { ph.add(EV_NEE, k, (uint32_t)e2 | (2u << 16)); return; }
  double area = pd->elem_width * pd->elem_height;
  T amp = w * f.Ar * (kd / PI) * cos_o * (area * cos_el / (r * r)) * (double)pd->n_elem * fd;
  T tof = t;
  V3<T> p = x;
  T remaining = r;
  int reg = region;
  int crossings = 0;
  for (;;) {
    Hit<T> h = closest_hit(m, p, we, false);
    ++*segs;
    if (h.kind == HIT_NONE || val(h.t) >= val(remaining)) {
      tof = tof + remaining / m.c[reg];
      amp = amp * exp(-(m.a[reg] * remaining));
      break;
    }
    tof = tof + h.t / m.c[reg];
    amp = amp * exp(-(m.a[reg] * h.t));
    remaining = remaining - h.t;
    p = p + we * h.t;
    V3<T> n; int other; double kd2;
    surface_at(m, h, p, reg, &n, &other, &kd2);
    Interface<T> g = interface_at(we, n, m.c[reg], m.Z[reg], m.c[other], m.Z[other]);
    ++crossings;
    if (g.tir) { ph.add(EV_NEE, k, (uint32_t)e2 | (3u << 16) | ((uint32_t)crossings << 20)); return; }
    amp = amp * g.At;
    reg = other;
  }
  ph.add(EV_NEE, k, (uint32_t)e2 | ((uint32_t)crossings << 20));
  sink.deposit(txi, e2, tof, amp, ray);
}

// One primary path (Sec. 2.3.1-2.3.4).
template <class T>
void trace_path(const Model<T>& m, Sink<T>& sink, int txi, int64_t ray, uint64_t* hash_out,
                int64_t* segs) {
  const OrProbeDesc* pd = m.pd;
  const OrRunDesc* rd = m.rd;
  PathHash ph;
  const uint32_t tx_id = rd->tx_ids[txi];
  const double th = rd->angles[txi];
  const int e_emit = (int)(ray / rd->rays_per_elem);

  // Emission (Sec. 2.3.1): origin uniform over the element face; direction is
  // the steering direction (reading: a plane-wave transmit emits parallel
  // rays); the transmit delay enters only as a time stamp; weight f_d / N with
  // f_d = max(0, n . w0) (Eq. directivity) and N rays per element.
  U4 u = draw(rd->seed, (uint64_t)ray, tx_id, 0);
  double xe = (e_emit - 0.5 * (pd->n_elem - 1)) * pd->pitch;
  V3<T> o{T(xe + (u.u[0] - 0.5) * pd->elem_width), T((u.u[1] - 0.5) * pd->elem_height), T(0.0)};
  V3<T> w{T(std::sin(th)), T(0.0), T(std::cos(th))};
  T t = o.x * (std::sin(th) / pd->c_ref);
  T wt = T(std::max(0.0, std::cos(th)) / rd->rays_per_elem);
  int region = m.sd->start_region;
  bool last_delta = true;

  for (int k = 1;; ++k) {
    Hit<T> h = closest_hit(m, o, w, true);
    ++*segs;
    ph.add(EV_HIT, k, ((uint32_t)h.kind << 24) | ((uint32_t)(h.index + 1) & 0xFFFFFFu));
    if (h.kind == HIT_NONE) break;          // escapes the scene
    // travel time and attenuation along the segment
    t = t + h.t / m.c[region];
    wt = wt * exp(-(m.a[region] * h.t));
    V3<T> x = o + w * h.t;
    if (h.kind == HIT_ARRAY) {
      // A path that reaches the array face deposits its pressure on the
      // element it lands on, weighted by the receive directivity. Paths whose
      // last event was diffuse are already counted by the secondary rays
      // (each path is counted once).
      double half_w = 0.5 * pd->n_elem * pd->pitch;
      bool counted = (last_delta || rd->nee_mode == 1) && std::fabs(val(x.x)) < half_w &&
                     std::fabs(val(x.y)) < 0.5 * pd->elem_height;
      if (counted) {
        int e = (int)std::floor((val(x.x) + half_w) / pd->pitch);
        e = std::min(std::max(e, 0), pd->n_elem - 1);
        T fd = directivity(pd, -w.z);
        ph.add(EV_ARRAY, k, (uint32_t)e);
        if (val(fd) > 0.0) sink.deposit(txi, e, t, wt * fd, ray);
      } else {
        ph.add(EV_ARRAY, k, 0xFFFFFFu);
      }
      break;
    }
    if (k > rd->max_bounces) break;         // only an array hit counts after the last interaction

    V3<T> n; int other; double kd; T rho;
    surface_at(m, h, x, region, &n, &other, &kd, &rho);
    Interface<T> f = interface_at(w, n, m.c[region], m.Z[region], m.c[other], m.Z[other]);
    U4 v = draw(rd->seed, (uint64_t)ray, tx_id, (uint32_t)k);

    if (kd > 0.0 && rd->nee_mode == 0) {
      int e2 = std::min((int)(v.u[3] * pd->n_elem), pd->n_elem - 1);
      receiver_ray(m, sink, ph, segs, txi, ray, k, region, x, f, kd, wt, t, e2);
    }

    // Branch on the energy split (reading: weights carry pressure; the choice
    // is made by energy, and the weight is multiplied by the pressure
    // coefficient over the choice probability, which is a sampling density
    // and is not differentiated).
    double RE = f.RE;
    if (rd->prob_mode != 0) {
      double* slot = rd->prob_buf +
                     ((int64_t)txi * rd->ray_count + (ray - rd->ray_begin)) * rd->max_bounces + (k - 1);
      if (rd->prob_mode == 1) *slot = RE; else RE = *slot;
    }
    double p_spec = (1.0 - kd) * RE;
    uint32_t branch;
    bool ends = false;
    if (v.u[0] < p_spec) {
      // glossy about a GGX microfacet (the mirror when rho = 0); a glossy
      // path deposits on the array like a specular one
      Glossy<T> gl = glossy_reflect(w, f, rho, v.u[1], v.u[2]);
      w = gl.dir;
      wt = wt * f.Ar / RE * gl.g;
      ends = !gl.ok;
      last_delta = true; branch = ends ? 3 : 0;
    } else if (v.u[0] < RE) {
      w = cosine_dir(f.n_r, v.u[1], v.u[2]);
      wt = wt * f.Ar / RE;
      last_delta = false; branch = 1;
    } else {
      T eta = m.c[other] / m.c[region];
      w = refract_dir(w, f, eta);
      wt = wt * f.At / (1.0 - RE);
      region = other;
      last_delta = true; branch = 2;
    }
    ph.add(EV_BRANCH, k, branch | (f.tir ? 0x10u : 0u));
    if (ends) break;
    o = x;
  }
  if (hash_out) *hash_out = ph.h;
}

// amplitude attenuation coefficient [Np/m] from alpha [dB/cm/MHz] at f0
// (reading: evaluated at the centre frequency, no dispersion).
inline double np_per_m(double f0) { return (f0 * 1e-6) * 100.0 * std::log(10.0) / 20.0; }

// Scene parameters theta -> model; for the dual model, parameter sel[i]
// carries tangent direction i.
template <class T>
void build_model(Model<T>& m, const OrSceneDesc* sd, const OrProbeDesc* pd, const OrRunDesc* rd,
                 const std::vector<T>& th) {
  m.sd = sd; m.pd = pd; m.rd = rd;
  m.c.resize(sd->n_regions); m.Z.resize(sd->n_regions); m.a.resize(sd->n_regions);
  double k = np_per_m(pd->f0);
  for (int r = 0; r < sd->n_regions; ++r) {
    m.c[r] = th[3 * r]; m.Z[r] = th[3 * r + 1]; m.a[r] = th[3 * r + 2] * k;
  }
  int off = 3 * sd->n_regions;
  for (int p = 0; p < sd->n_planes; ++p) m.pz.push_back(th[off + p]);
  off += sd->n_planes;
  for (int s = 0; s < sd->n_spheres; ++s) {
    m.sc.push_back({th[off + 4 * s], th[off + 4 * s + 1], th[off + 4 * s + 2]});
    m.sr.push_back(th[off + 4 * s + 3]);
  }
  off += 4 * sd->n_spheres;
  for (int c = 0; c < sd->n_cylinders; ++c) {
    m.ccx.push_back(th[off + 3 * c]); m.ccz.push_back(th[off + 3 * c + 1]); m.cr.push_back(th[off + 3 * c + 2]);
  }
  off += 3 * sd->n_cylinders;
  for (int p = 0; p < sd->n_planes; ++p) m.rho_p.push_back(th[off + p]);
  off += sd->n_planes;
  for (int s = 0; s < sd->n_spheres; ++s) m.rho_s.push_back(th[off + s]);
  off += sd->n_spheres;
  for (int c = 0; c < sd->n_cylinders; ++c) m.rho_c.push_back(th[off + c]);
  off += sd->n_cylinders;
  for (int j = 0; j < sd->n_meshes; ++j) m.rho_m.push_back(th[off + j]);
  off += sd->n_meshes;
  if (sd->n_meshes > 0) {
    for (int j = 0; j < sd->n_meshes * sd->n_basis; ++j) m.q.push_back(th[off + j]);
    m.vpos.resize(3 * sd->n_vertices);
    for (int64_t v = 0; v < sd->n_vertices; ++v) {
      V3<T> p = vertex(m, (int)v);
      m.vpos[3 * v] = val(p.x); m.vpos[3 * v + 1] = val(p.y); m.vpos[3 * v + 2] = val(p.z);
    }
    m.bvh.build(m.vpos, sd->tris, sd->n_triangles);
  }
}

// theta = [(c, Z, alpha) per region, plane depths, (x, y, z, r) per sphere,
//          (x, z, R) per cylinder, roughness per plane, sphere, cylinder and
//          mesh, mesh basis coefficients]
int n_params_of(const OrSceneDesc* sd) {
  return 3 * sd->n_regions + sd->n_planes + 4 * sd->n_spheres + 3 * sd->n_cylinders +
         (sd->n_planes + sd->n_spheres + sd->n_cylinders + sd->n_meshes) + sd->n_meshes * sd->n_basis;
}

struct Result {
  std::vector<OrContrib> contribs;
  std::vector<double> g_theta;
  int64_t segments = 0;
};

}  // namespace

extern "C" {

// Traces rays [ray_begin, ray_begin + ray_count) of every transmit.
// Returns an opaque result handle (contributions in ray order), or NULL on bad
// arguments. If g_h is non-NULL, also accumulates d L / d theta[sel[i]] for
// i < n_sel (n_sel <= 64) into the result's gradient, given d L / d h = g_h
// ([n_tx][n_elem][n_t]). hashes (optional): [n_tx][ray_count] decision hashes.
void* oracle_trace(const OrSceneDesc* sd, const OrProbeDesc* pd, const OrRunDesc* rd,
                   const double* theta, const double* g_h, const int32_t* sel, int n_sel,
                   uint64_t* hashes) {
  if (!sd || !pd || !rd || !theta || rd->rays_per_elem <= 0 || rd->ray_count < 0) return nullptr;
  if (g_h && (n_sel < 0 || n_sel > MAXD)) return nullptr;
  if (rd->prob_mode != 0 && (!rd->prob_buf || rd->max_bounces <= 0)) return nullptr;
  const int64_t chunk = 1024;
  const int64_t n_ray = rd->ray_count;
  const int64_t n_chunks_tx = (n_ray + chunk - 1) / chunk;
  const int64_t n_chunks = n_chunks_tx * rd->n_tx;
  std::vector<std::vector<OrContrib>> parts(n_chunks);
  std::vector<std::vector<double>> gparts(g_h ? n_chunks : 0);
  std::vector<int64_t> segs(n_chunks, 0);
  if (rd->n_threads > 0) omp_set_num_threads(rd->n_threads);

  const int np = n_params_of(sd);
  for (int i = 0; g_h && i < n_sel; ++i) if (sel[i] < 0 || sel[i] >= np) return nullptr;
  Model<double> md;
  if (!g_h) build_model(md, sd, pd, rd, std::vector<double>(theta, theta + np));

#pragma omp parallel
  {
    Model<Dual> mg;
    if (g_h) {
      g_nd = n_sel;
      std::vector<Dual> th(np);
      for (int j = 0; j < np; ++j) th[j] = Dual(theta[j]);
      for (int i = 0; i < n_sel; ++i) th[sel[i]].d[i] = 1.0;
      build_model(mg, sd, pd, rd, th);
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_chunks; ++c) {
      int txi = (int)(c / n_chunks_tx);
      int64_t r0 = (c % n_chunks_tx) * chunk;
      int64_t r1 = std::min(n_ray, r0 + chunk);
      if (g_h) {
        gparts[c].assign(n_sel, 0.0);
        Sink<Dual> sink{&parts[c], g_h, pd, gparts[c].data()};
        for (int64_t r = r0; r < r1; ++r)
          trace_path(mg, sink, txi, rd->ray_begin + r, hashes ? hashes + txi * n_ray + r : nullptr,
                     &segs[c]);
      } else {
        Sink<double> sink{&parts[c]};
        for (int64_t r = r0; r < r1; ++r)
          trace_path(md, sink, txi, rd->ray_begin + r, hashes ? hashes + txi * n_ray + r : nullptr,
                     &segs[c]);
      }
    }
  }
  Result* res = new Result;
  size_t total = 0;
  for (auto& p : parts) total += p.size();
  res->contribs.reserve(total);
  for (auto& p : parts) res->contribs.insert(res->contribs.end(), p.begin(), p.end());
  if (g_h) {
    res->g_theta.assign(n_sel, 0.0);
    for (auto& g : gparts) for (int i = 0; i < n_sel; ++i) res->g_theta[i] += g[i];
  }
  for (auto s : segs) res->segments += s;
  return res;
}

int64_t oracle_result_count(void* h) { return h ? (int64_t)((Result*)h)->contribs.size() : -1; }
int64_t oracle_result_segments(void* h) { return h ? ((Result*)h)->segments : -1; }

// Copies the contributions (tx, elem, t, a, ray) and the gradient (if any).
void oracle_result_copy(void* h, int32_t* tx, int32_t* elem, double* t, double* a, int64_t* ray,
                        double* g_theta) {
  Result* r = (Result*)h;
  for (size_t i = 0; i < r->contribs.size(); ++i) {
    const OrContrib& c = r->contribs[i];
    if (tx) tx[i] = c.tx;
    if (elem) elem[i] = c.elem;
    if (t) t[i] = c.t;
    if (a) a[i] = c.a;
    if (ray) ray[i] = c.ray;
  }
  if (g_theta) for (size_t i = 0; i < r->g_theta.size(); ++i) g_theta[i] = r->g_theta[i];
}

void oracle_result_free(void* h) { delete (Result*)h; }

// Splats contributions into h[n_tx][n_elem][n_t] (Sec. 2.3.4): the deposit at
// time t goes to samples j0 = floor(t fs) and j0 + 1 with weights 1 - f and f.
void oracle_splat(int64_t n, const int32_t* tx, const int32_t* elem, const double* t,
                  const double* a, int n_elem, int n_t, double fs, double* h) {
  for (int64_t i = 0; i < n; ++i) {
    double x = t[i] * fs;
    double j0d = std::floor(x);
    double f = x - j0d;
    long j0 = (long)j0d;
    double* row = h + ((long)tx[i] * n_elem + elem[i]) * (long)n_t;
    if (j0 >= 0 && j0 < n_t) row[j0] += a[i] * (1.0 - f);
    if (j0 + 1 >= 0 && j0 + 1 < n_t) row[j0 + 1] += a[i] * f;
  }
}

// Exposed pieces for the oracle's own pins.
void oracle_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out) { philox4x64_10(ctr, key, out); }

double oracle_uniform(uint64_t x) { return uniform_from(x); }

// Interface physics for one incidence: outputs A_r, A_t, R_E, reflected and
// transmitted directions (the latter zero on total internal reflection).
void oracle_interface(const double* w, const double* n, double c1, double Z1, double c2, double Z2,
                      double* out_coef /*Ar, At, RE, tir*/, double* w_refl, double* w_trans) {
  V3<double> wv{w[0], w[1], w[2]}, nv{n[0], n[1], n[2]};
  Interface<double> f = interface_at(wv, nv, c1, Z1, c2, Z2);
  out_coef[0] = f.Ar; out_coef[1] = f.At; out_coef[2] = f.RE; out_coef[3] = f.tir ? 1.0 : 0.0;
  V3<double> r = reflect_dir(wv, f);
  w_refl[0] = r.x; w_refl[1] = r.y; w_refl[2] = r.z;
  if (f.tir) { w_trans[0] = w_trans[1] = w_trans[2] = 0.0; }
  else {
    V3<double> t = refract_dir(wv, f, c2 / c1);
    w_trans[0] = t.x; w_trans[1] = t.y; w_trans[2] = t.z;
  }
}

void oracle_cosine_dir(const double* n, double u1, double u2, double* out) {
  V3<double> d = cosine_dir(V3<double>{n[0], n[1], n[2]}, u1, u2);
  out[0] = d.x; out[1] = d.y; out[2] = d.z;
}

double oracle_directivity(const OrProbeDesc* pd, double cos_a) { return directivity(pd, cos_a); }

// Rough reflection of w at normal n between media (c1, Z1) and (c2, Z2):
// out = reflected direction (3), estimator factor g, ok flag.
void oracle_glossy(const double* w, const double* n, double c1, double Z1, double c2, double Z2,
                   double rho, double u1, double u2, double* out) {
  V3<double> wv{w[0], w[1], w[2]}, nv{n[0], n[1], n[2]};
  Interface<double> f = interface_at(wv, nv, c1, Z1, c2, Z2);
  Glossy<double> g = glossy_reflect(wv, f, rho, u1, u2);
  out[0] = g.dir.x; out[1] = g.dir.y; out[2] = g.dir.z; out[3] = g.g; out[4] = g.ok ? 1.0 : 0.0;
}

}  // extern "C"
