// C-ABI of the library (declared in include/usrt.h): argument checks on the
// host, workspace slicing, and the launch sequence of each entry point.
#include "usrt.h"

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fir.h"
#include "kernels.h"

using namespace usrt;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define US_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(US_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define US_CHECK(cond, msg)                    \
  do {                                         \
    if (!(cond)) return fail(US_EINVAL, msg);  \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Carves aligned sub-buffers out of a workspace.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T> T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

}  // namespace

// Optional per-kernel timing: event pairs recorded around launches.
struct ProfileLog {
  bool on = false;
  struct Pending { std::string name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<std::string, std::pair<double, long>>> totals;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

struct us_ctx {
  int device;
  ProfileLog prof;
};

// Scratch of us_beamform_static, the entry point for callers that cannot
// allocate: the analytic signal of the channels, at most kStaticScratchBytes
// (64 MiB, 8,388,608 complex samples). Every GPU that loads the library holds
// its own copy of the array until the process ends. In host code the array's
// name is not a device address: us_create looks up each device's copy once
// (hipGetSymbolAddress with that device current) and every use goes through
// the pointer kept here.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace {

// Brackets the launches issued in its scope with events when profiling is on.
struct Timed {
  ProfileLog* log;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  // a null name records nothing (the allocation-free entry point)
  Timed(us_ctx* ctx, const char* n, hipStream_t st) : log(&ctx->prof), name(n), s(st) {
    if (log->on && n) { a = log->get(); (void)hipEventRecord(a, s); }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = log->get();
    (void)hipEventRecord(b, s);
    log->pending.push_back({name, a, b});
  }
};

}  // namespace

// Destroys a half-built handle when an upload returns early (the US_HIP
// checks of its copies); release() hands the finished handle to the caller.
template <class T, int (*Destroy)(T*)>
struct UploadGuard {
  T* h;
  ~UploadGuard() { if (h) Destroy(h); }
  T* release() { T* t = h; h = nullptr; return t; }
};

struct us_probe {
  us_ctx* ctx;
  int device;   // kept for destroy, which must not read the context
  us_probe_desc d;
  ProbeView pv;
  int M;
  float* taps;          // s[m], m = -M..M
  float* taps_rev;      // s[-m]
  float* dtaps_rev;     // d s[-m] / d f0
  float2* twiddle;      // exp(-2 pi i j / n_t), j < n_t / 2 (power-of-two n_t only)
};

struct us_scene {
  us_ctx* ctx;
  int device;   // kept for destroy, which must not read the context
  int n_regions, n_planes, n_spheres, start_region, n_params;
  bool any_diffuse;
  double* theta;
  int* plane_regions;
  double* plane_kd;
  int* sphere_regions;
  double* sphere_kd;
  int n_cylinders;
  int* cylinder_regions;
  double* cylinder_kd;
  // meshes
  int n_meshes, n_basis, q_offset, stack_cap;
  int* mesh_regions;
  double* mesh_kd;
  int* tri_orig;
  MeshDevice mesh;   // owns vrest, vnormal, vbasis, vmesh, vcur, nodes, tri
  // bumped by us_scene_set_params: records of a recorded forward hold for
  // the parameters they were made with
  uint64_t version;
  // the last recorded forward on this scene (workspace and arguments), which
  // a recorded backward must match
  struct {
    const void* ws;
    uint64_t version;
    const us_probe* probe;
    uint64_t seed, tx_hash;
    int64_t ray_begin, ray_count;
    int32_t rays_per_elem, max_bounces, n_tx;
  } rec;
};

// Makes the device current and clears the runtime's last error, so that a
// failure left by an unrelated earlier HIP call of this thread (the caller's,
// or a destroy's) is not reported as this call's.
static hipError_t bind_device(int device) {
  const hipError_t e = hipSetDevice(device);
  (void)hipGetLastError();
  return e;
}

extern "C" {

const char* us_last_error(void) { return g_err.c_str(); }

int us_create(int device, us_ctx** out) {
  US_CHECK(out != nullptr, "us_create: out is NULL");
  int n = 0;
  US_HIP(hipGetDeviceCount(&n));
  US_CHECK(device >= 0 && device < n, "us_create: no such device");
  US_HIP(bind_device(device));
  if (device < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      void* p = nullptr;
      US_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      g_scratch_ptr[device] = p;
    }
  }
  *out = new us_ctx{device};
  return US_OK;
}

int us_destroy(us_ctx* ctx) {
  delete ctx;
  return US_OK;
}

int us_probe_upload(us_ctx* ctx, const us_probe_desc* d, us_probe** out) {
  US_CHECK(ctx && d && out, "us_probe_upload: NULL argument");
  US_CHECK(d->n_elem >= 1 && d->n_elem <= 65535, "us_probe_upload: n_elem must be in [1, 65535]");
  US_CHECK(d->pitch > 0 && d->elem_width > 0 && d->elem_height > 0, "us_probe_upload: element geometry must be positive");
  US_CHECK(d->f0 > 0 && d->n_cycles > 0 && d->fs > 0 && d->c_ref > 0, "us_probe_upload: f0, n_cycles, fs, c_ref must be positive");
  US_CHECK(d->n_t >= 2 && d->n_t <= (1 << 20), "us_probe_upload: n_t must be in [2, 2^20]");
  US_CHECK(d->alpha_main >= 0 && d->alpha_main < d->alpha_cut && d->alpha_cut <= M_PI, "us_probe_upload: need 0 <= alpha_main < alpha_cut <= pi");
  // Eq. axial_sig: envelope FWHM n_cycles / f0; taps until the envelope falls to 1e-7
  const double sigma = std::pow(d->n_cycles / (2.0 * d->f0), 2) / std::log(2.0);
  const int M = (int)std::ceil(d->fs * std::sqrt(sigma * std::log(1e7)));
  US_CHECK(M >= 0 && M <= 511, "us_probe_upload: pulse longer than 1023 taps");
  std::vector<float> taps(2 * M + 1), rev(2 * M + 1), drev(2 * M + 1);
  for (int m = -M; m <= M; ++m) {
    const double t = m / d->fs;
    const double env = std::exp(-t * t / sigma), w = 2.0 * M_PI * d->f0 * t;
    taps[m + M] = (float)(std::sin(w) * env);
    // sigma scales as 1 / f0^2, so d env / d f0 = -env 2 t^2 / (sigma f0)
    drev[M - m] = (float)(2.0 * M_PI * t * std::cos(w) * env - std::sin(w) * env * 2.0 * t * t / (sigma * d->f0));
  }
  for (int i = 0; i < 2 * M + 1; ++i) rev[i] = taps[2 * M - i];
  US_HIP(bind_device(ctx->device));
  us_probe* p = new us_probe{};
  UploadGuard<us_probe, us_probe_destroy> guard{p};
  p->ctx = ctx;
  p->device = ctx->device;
  p->d = *d;
  p->M = M;
  p->pv = ProbeView{d->n_elem, d->n_t, d->pitch, d->elem_width, d->elem_height, d->f0, d->fs,
                    d->c_ref, d->alpha_main, d->alpha_cut, std::cos(d->alpha_main), std::cos(d->alpha_cut)};
  const bool pow2 = (d->n_t & (d->n_t - 1)) == 0;
  if (hipMalloc(&p->taps, taps.size() * sizeof(float)) != hipSuccess ||
      hipMalloc(&p->taps_rev, rev.size() * sizeof(float)) != hipSuccess ||
      hipMalloc(&p->dtaps_rev, drev.size() * sizeof(float)) != hipSuccess ||
      (pow2 && hipMalloc(&p->twiddle, (d->n_t / 2) * sizeof(float2)) != hipSuccess))
    return fail(US_ENOMEM, "us_probe_upload: hipMalloc failed");
  US_HIP(hipMemcpy(p->taps, taps.data(), taps.size() * sizeof(float), hipMemcpyHostToDevice));
  US_HIP(hipMemcpy(p->taps_rev, rev.data(), rev.size() * sizeof(float), hipMemcpyHostToDevice));
  US_HIP(hipMemcpy(p->dtaps_rev, drev.data(), drev.size() * sizeof(float), hipMemcpyHostToDevice));
  if (pow2) {
    std::vector<float2> tw(d->n_t / 2);
    for (int j = 0; j < d->n_t / 2; ++j) {
      const double ang = -2.0 * M_PI * j / d->n_t;
      tw[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    US_HIP(hipMemcpy(p->twiddle, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  }
  *out = guard.release();
  return US_OK;
}

int us_probe_destroy(us_probe* p) {
  if (!p) return US_OK;
  (void)hipSetDevice(p->device);
  (void)hipFree(p->taps);
  (void)hipFree(p->taps_rev);
  (void)hipFree(p->dtaps_rev);
  (void)hipFree(p->twiddle);
  delete p;
  return US_OK;
}

int us_scene_upload(us_ctx* ctx, const us_scene_desc* d, us_scene** out, int32_t* n_params) {
  US_CHECK(ctx && d && out && d->theta, "us_scene_upload: NULL argument");
  US_CHECK(d->n_regions >= 1 && d->n_regions <= kMaxRegions, "us_scene_upload: n_regions must be in [1, 64]");
  US_CHECK(d->n_planes >= 0 && d->n_planes <= kMaxPlanes, "us_scene_upload: at most 16 planes");
  US_CHECK(d->n_spheres >= 0 && d->n_spheres <= kMaxSpheres, "us_scene_upload: at most 32 spheres");
  US_CHECK(d->n_planes == 0 || (d->plane_regions && d->plane_kd), "us_scene_upload: plane arrays missing");
  US_CHECK(d->n_spheres == 0 || (d->sphere_regions && d->sphere_kd), "us_scene_upload: sphere arrays missing");
  US_CHECK(d->n_cylinders >= 0 && d->n_cylinders <= kMaxCylinders, "us_scene_upload: at most 16 cylinders");
  US_CHECK(d->n_cylinders == 0 || (d->cylinder_regions && d->cylinder_kd),
           "us_scene_upload: cylinder arrays missing");
  US_CHECK(d->start_region >= 0 && d->start_region < d->n_regions, "us_scene_upload: start_region out of range");
  US_CHECK(d->n_meshes >= 0 && d->n_meshes <= kMaxMeshes, "us_scene_upload: at most 32 meshes");
  const int nm = d->n_meshes;
  if (nm > 0) {
    US_CHECK(d->n_basis >= 0 && d->n_basis <= 4096, "us_scene_upload: n_basis must be in [0, 4096]");
    US_CHECK(d->mesh_regions && d->mesh_kd && d->vertices && d->vnormal && d->vmesh && d->triangles &&
                 d->tmesh && (d->n_basis == 0 || d->vbasis),
             "us_scene_upload: mesh arrays missing");
    US_CHECK(d->n_vertices >= 3 && d->n_vertices < (1L << 30), "us_scene_upload: n_vertices must be in [3, 2^30)");
    US_CHECK(d->n_triangles >= 1 && d->n_triangles < (1L << 27), "us_scene_upload: n_triangles must be in [1, 2^27)");
  }
  // theta = [regions, plane depths, spheres, cylinders, roughness (planes,
  // spheres, cylinders, meshes), mesh basis coefficients]
  const int nc = d->n_cylinders;
  const int cyl_offset = 3 * d->n_regions + d->n_planes + 4 * d->n_spheres;
  const int rough_offset = cyl_offset + 3 * nc;
  const int q_offset = rough_offset + d->n_planes + d->n_spheres + nc + nm;
  const int np = q_offset + (nm > 0 ? nm * d->n_basis : 0);
  for (int k = 0; k < d->n_planes + d->n_spheres + nc + nm; ++k)
    US_CHECK(d->theta[rough_offset + k] >= 0 && std::isfinite(d->theta[rough_offset + k]),
             "us_scene_upload: roughness must be finite and >= 0");
  for (int r = 0; r < d->n_regions; ++r)
    US_CHECK(d->theta[3 * r] > 0 && d->theta[3 * r + 1] > 0 && d->theta[3 * r + 2] >= 0,
             "us_scene_upload: region needs c > 0, Z > 0, alpha >= 0");
  bool diffuse = false;
  for (int k = 0; k < d->n_planes; ++k) {
    for (int j = 0; j < 2; ++j)
      US_CHECK(d->plane_regions[2 * k + j] >= 0 && d->plane_regions[2 * k + j] < d->n_regions, "us_scene_upload: plane region out of range");
    US_CHECK(d->plane_kd[k] >= 0 && d->plane_kd[k] <= 1, "us_scene_upload: kd must be in [0, 1]");
    diffuse |= d->plane_kd[k] > 0;
  }
  for (int k = 0; k < d->n_spheres; ++k) {
    for (int j = 0; j < 2; ++j)
      US_CHECK(d->sphere_regions[2 * k + j] >= 0 && d->sphere_regions[2 * k + j] < d->n_regions, "us_scene_upload: sphere region out of range");
    US_CHECK(d->sphere_kd[k] >= 0 && d->sphere_kd[k] <= 1, "us_scene_upload: kd must be in [0, 1]");
    US_CHECK(d->theta[3 * d->n_regions + d->n_planes + 4 * k + 3] > 0, "us_scene_upload: sphere radius must be positive");
    diffuse |= d->sphere_kd[k] > 0;
  }
  for (int k = 0; k < nc; ++k) {
    for (int j = 0; j < 2; ++j)
      US_CHECK(d->cylinder_regions[2 * k + j] >= 0 && d->cylinder_regions[2 * k + j] < d->n_regions,
               "us_scene_upload: cylinder region out of range");
    US_CHECK(d->cylinder_kd[k] >= 0 && d->cylinder_kd[k] <= 1, "us_scene_upload: kd must be in [0, 1]");
    US_CHECK(d->theta[cyl_offset + 3 * k + 2] > 0, "us_scene_upload: cylinder radius must be positive");
    diffuse |= d->cylinder_kd[k] > 0;
  }
  MeshHierarchy H;
  const long nv = nm > 0 ? (long)d->n_vertices : 0, nt = nm > 0 ? (long)d->n_triangles : 0;
  const int nb = nm > 0 ? d->n_basis : 0;
  if (nm > 0) {
    for (int m = 0; m < nm; ++m) {
      for (int j = 0; j < 2; ++j)
        US_CHECK(d->mesh_regions[2 * m + j] >= 0 && d->mesh_regions[2 * m + j] < d->n_regions, "us_scene_upload: mesh region out of range");
      US_CHECK(d->mesh_kd[m] >= 0 && d->mesh_kd[m] <= 1, "us_scene_upload: kd must be in [0, 1]");
      diffuse |= d->mesh_kd[m] > 0;
    }
    for (long v = 0; v < nv; ++v) {
      US_CHECK(d->vmesh[v] >= 0 && d->vmesh[v] < nm, "us_scene_upload: vmesh out of range");
      US_CHECK(v == 0 || d->vmesh[v] >= d->vmesh[v - 1],
               "us_scene_upload: vertices must be concatenated in mesh order");
      for (int k = 0; k < 3; ++k)
        US_CHECK(std::isfinite(d->vertices[3 * v + k]) && std::isfinite(d->vnormal[3 * v + k]),
                 "us_scene_upload: vertices and vnormal must be finite");
    }
    for (long t = 0; t < nt; ++t) {
      const int32_t* tv = d->triangles + 3 * t;
      US_CHECK(d->tmesh[t] >= 0 && d->tmesh[t] < nm, "us_scene_upload: tmesh out of range");
      for (int j = 0; j < 3; ++j)
        US_CHECK(tv[j] >= 0 && tv[j] < nv && d->vmesh[tv[j]] == d->tmesh[t],
                 "us_scene_upload: triangle vertex out of range or of another mesh");
      const double* a = d->vertices + 3 * (long)tv[0];
      const double* b = d->vertices + 3 * (long)tv[1];
      const double* c = d->vertices + 3 * (long)tv[2];
      const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                   cz = e1[0] * e2[1] - e1[1] * e2[0];
      US_CHECK(cx * cx + cy * cy + cz * cz > 0.0, "us_scene_upload: zero-area triangle");
    }
    US_CHECK(build_mesh_bvh(d->vertices, nv, d->triangles, d->tmesh, nt, H) == 0,
             "us_scene_upload: mesh hierarchy too deep (degenerate triangle set)");
  }
  US_HIP(bind_device(ctx->device));
  us_scene* s = new us_scene{};
  UploadGuard<us_scene, us_scene_destroy> guard{s};
  s->ctx = ctx;
  s->device = ctx->device;
  s->n_regions = d->n_regions; s->n_planes = d->n_planes; s->n_spheres = d->n_spheres;
  s->n_cylinders = nc;
  s->start_region = d->start_region; s->n_params = np; s->any_diffuse = diffuse;
  s->n_meshes = nm; s->n_basis = nb; s->q_offset = q_offset; s->stack_cap = nm > 0 ? 3 * H.depth : 0;
  bool ok = hipMalloc(&s->theta, np * sizeof(double)) == hipSuccess &&
            hipMalloc(&s->plane_regions, (2 * d->n_planes + 1) * sizeof(int)) == hipSuccess &&
            hipMalloc(&s->plane_kd, (d->n_planes + 1) * sizeof(double)) == hipSuccess &&
            hipMalloc(&s->sphere_regions, (2 * d->n_spheres + 1) * sizeof(int)) == hipSuccess &&
            hipMalloc(&s->sphere_kd, (d->n_spheres + 1) * sizeof(double)) == hipSuccess &&
            hipMalloc(&s->cylinder_regions, (2 * nc + 1) * sizeof(int)) == hipSuccess &&
            hipMalloc(&s->cylinder_kd, (nc + 1) * sizeof(double)) == hipSuccess &&
            hipMalloc(&s->mesh_regions, (2 * nm + 1) * sizeof(int)) == hipSuccess &&
            hipMalloc(&s->mesh_kd, (nm + 1) * sizeof(double)) == hipSuccess;
  MeshDevice& md = s->mesh;
  if (ok && nm > 0) {
    md.n_vertices = nv; md.n_triangles = nt; md.n_basis = nb;
    md.level_begin = H.level_begin;
    double *vrest = nullptr, *vnormal = nullptr, *vbasis = nullptr;
    int* vmesh = nullptr;
    int4* tri = nullptr;
    long* vbeg = nullptr;
    ok = hipMalloc(&vrest, 3 * nv * sizeof(double)) == hipSuccess &&
         hipMalloc(&vnormal, 3 * nv * sizeof(double)) == hipSuccess &&
         hipMalloc(&vbasis, (nv * nb + 1) * sizeof(double)) == hipSuccess &&
         hipMalloc(&vmesh, nv * sizeof(int)) == hipSuccess &&
         hipMalloc(&md.vcur, 3 * nv * sizeof(double)) == hipSuccess &&
         hipMalloc(&md.trec, nt * sizeof(TriRec)) == hipSuccess &&
         hipMalloc(&md.nodes, H.nodes.size() * sizeof(BvhNode)) == hipSuccess &&
         hipMalloc(&tri, nt * sizeof(int4)) == hipSuccess &&
         hipMalloc(&s->tri_orig, nt * sizeof(int)) == hipSuccess &&
         hipMalloc(&vbeg, (nm + 1) * sizeof(long)) == hipSuccess;
    md.vrest = vrest; md.vnormal = vnormal; md.vbasis = vbasis; md.vmesh = vmesh; md.tri = tri;
    md.vbeg = vbeg;
  }
  if (!ok) return fail(US_ENOMEM, "us_scene_upload: hipMalloc failed");
  if (nm > 0) {
    US_HIP(hipMemcpy(s->mesh_regions, d->mesh_regions, 2 * nm * sizeof(int), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy(s->mesh_kd, d->mesh_kd, nm * sizeof(double), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy((void*)md.vrest, d->vertices, 3 * nv * sizeof(double), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy((void*)md.vnormal, d->vnormal, 3 * nv * sizeof(double), hipMemcpyHostToDevice));
    if (nb > 0) US_HIP(hipMemcpy((void*)md.vbasis, d->vbasis, nv * nb * sizeof(double), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy((void*)md.vmesh, d->vmesh, nv * sizeof(int), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy(md.nodes, H.nodes.data(), H.nodes.size() * sizeof(BvhNode), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy((void*)md.tri, H.tri.data(), nt * sizeof(int4), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy(s->tri_orig, H.tri_orig.data(), nt * sizeof(int), hipMemcpyHostToDevice));
    std::vector<long> vb(nm + 1, nv);
    for (long v = nv - 1; v >= 0; --v) vb[d->vmesh[v]] = v;
    for (int m = nm - 1; m >= 0; --m) vb[m] = std::min(vb[m], vb[m + 1]);   // meshes without vertices
    US_HIP(hipMemcpy((void*)md.vbeg, vb.data(), (nm + 1) * sizeof(long), hipMemcpyHostToDevice));
  }
  US_HIP(hipMemcpy(s->theta, d->theta, np * sizeof(double), hipMemcpyHostToDevice));
  if (d->n_planes) {
    US_HIP(hipMemcpy(s->plane_regions, d->plane_regions, 2 * d->n_planes * sizeof(int), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy(s->plane_kd, d->plane_kd, d->n_planes * sizeof(double), hipMemcpyHostToDevice));
  }
  if (d->n_spheres) {
    US_HIP(hipMemcpy(s->sphere_regions, d->sphere_regions, 2 * d->n_spheres * sizeof(int), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy(s->sphere_kd, d->sphere_kd, d->n_spheres * sizeof(double), hipMemcpyHostToDevice));
  }
  if (nc) {
    US_HIP(hipMemcpy(s->cylinder_regions, d->cylinder_regions, 2 * nc * sizeof(int), hipMemcpyHostToDevice));
    US_HIP(hipMemcpy(s->cylinder_kd, d->cylinder_kd, nc * sizeof(double), hipMemcpyHostToDevice));
  }
  if (nm > 0) {
    launch_mesh_refit(md, s->theta + q_offset, nullptr);
    US_HIP(hipGetLastError());
    US_HIP(hipDeviceSynchronize());
  }
  *out = guard.release();
  if (n_params) *n_params = np;
  return US_OK;
}

int us_scene_destroy(us_scene* s) {
  if (!s) return US_OK;
  (void)hipSetDevice(s->device);
  (void)hipFree(s->theta);
  (void)hipFree(s->plane_regions);
  (void)hipFree(s->plane_kd);
  (void)hipFree(s->sphere_regions);
  (void)hipFree(s->sphere_kd);
  (void)hipFree(s->cylinder_regions);
  (void)hipFree(s->cylinder_kd);
  (void)hipFree(s->mesh_regions);
  (void)hipFree(s->mesh_kd);
  (void)hipFree(s->tri_orig);
  (void)hipFree((void*)s->mesh.vrest);
  (void)hipFree((void*)s->mesh.vnormal);
  (void)hipFree((void*)s->mesh.vbasis);
  (void)hipFree((void*)s->mesh.vmesh);
  (void)hipFree(s->mesh.vcur);
  (void)hipFree(s->mesh.trec);
  (void)hipFree(s->mesh.nodes);
  (void)hipFree((void*)s->mesh.tri);
  (void)hipFree((void*)s->mesh.vbeg);
  delete s;
  return US_OK;
}

int us_scene_set_params(us_scene* s, const double* theta_dev, int32_t n_params, void* stream) {
  US_CHECK(s && theta_dev, "us_scene_set_params: NULL argument");
  US_CHECK(n_params == s->n_params, "us_scene_set_params: n_params does not match the scene");
  US_HIP(bind_device(s->ctx->device));
  US_HIP(hipMemcpyAsync(s->theta, theta_dev, n_params * sizeof(double), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  ++s->version;
  if (s->n_meshes > 0) {
    launch_mesh_refit(s->mesh, s->theta + s->q_offset, (hipStream_t)stream);
    US_HIP(hipGetLastError());
  }
  return US_OK;
}

}  // extern "C"

namespace {

SceneView scene_view(const us_scene* s, const us_probe* p) {
  SceneView v{};
  v.theta = s->theta;
  v.plane_regions = s->plane_regions;
  v.plane_kd = s->plane_kd;
  v.sphere_regions = s->sphere_regions;
  v.sphere_kd = s->sphere_kd;
  v.n_cylinders = s->n_cylinders;
  v.cylinder_regions = s->cylinder_regions;
  v.cylinder_kd = s->cylinder_kd;
  v.n_regions = s->n_regions;
  v.n_planes = s->n_planes;
  v.n_spheres = s->n_spheres;
  v.start_region = s->start_region;
  v.n_meshes = s->n_meshes;
  v.n_basis = s->n_basis;
  v.stack_cap = s->stack_cap;
  v.mesh_regions = s->mesh_regions;
  v.mesh_kd = s->mesh_kd;
  v.nodes = s->mesh.nodes;
  v.trec = s->mesh.trec;
  v.tri = s->mesh.tri;
  v.tri_orig = s->tri_orig;
  v.vcur = s->mesh.vcur;
  v.vnormal = s->mesh.vnormal;
  v.vbasis = s->mesh.vbasis;
  // amplitude attenuation at f0: alpha [dB/cm/MHz] * f0 [MHz] * 100 cm/m / (20 / ln 10)
  v.np_per_m = (p->d.f0 * 1e-6) * 100.0 * std::log(10.0) / 20.0;
  return v;
}

int fill_tx(TxTable& t, const us_tx_desc* tx, int first, int count) {
  std::memset(&t, 0, sizeof(t));
  t.n = count;
  for (int i = 0; i < count; ++i) {
    const double a = tx[first + i].angle;
    if (!(std::fabs(a) < 0.5 * M_PI)) return -1;
    t.sin_a[i] = std::sin(a);
    t.cos_a[i] = std::cos(a);
    t.id[i] = tx[first + i].id;
  }
  return 0;
}

// Rays per chunk when the caller sizes the workspace with
// us_simulate_rf_workspace_size (about 200 bytes of queue per ray).
constexpr long kDefaultChunk = 1L << 24;

// Deposits recorded for the binned splat per ray of a chunk (more spill to
// direct atomics).
constexpr long kDepositsPerRay = 2;

// Rows of the widest transmit group when their deposits can be binned, else 0.
int bin_rows(int n_tx, const us_probe* p) {
  const long rows = (long)std::min(n_tx, kMaxTxPerLaunch) * p->d.n_elem;
  return rows <= kMaxBinRows && p->d.n_t < kMaxBinSamples ? (int)rows : 0;
}

// Keys of the receiver-segment sort: origin cell, target element.
long sort_keys(const us_probe* p) { return (long)p->d.n_elem * kSortCellsZ * kSortCellsX; }

// The origin cells span twice the aperture either side of its centre and
// the depth the record reaches at c_ref.
SegSort seg_sort(const us_probe* p) {
  const us_probe_desc& d = p->d;
  const double half = 0.5 * d.n_elem * d.pitch;
  const double depth = 0.5 * d.n_t / d.fs * d.c_ref;
  return SegSort{(int)sort_keys(p), d.n_elem, -2.0 * half, kSortCellsX / (4.0 * half), kSortCellsZ / depth};
}

// Scenes with meshes march their receiver segments in key order.
bool sorts_segments(const us_scene* scene) { return scene->n_meshes > 0 && scene->any_diffuse; }

size_t trace_fixed_bytes(int n_tx, const us_probe* p, int max_bounces, bool sorts) {
  Carver c{nullptr};
  c.take<long long>((size_t)n_tx * p->d.n_elem * p->d.n_t);
  c.take<unsigned long long>((size_t)max_bounces + 5 + kDepShards);
  const int rows = bin_rows(n_tx, p);
  if (rows > 0) c.take<char>(splat_scratch_bytes(rows));
  if (sorts) {
    c.take<uint32_t>((size_t)sort_keys(p));
    c.take<uint32_t>((size_t)kSortBlocks);
  }
  return c.off;
}

size_t trace_per_ray_bytes() { return 2 * kRayQueueBytesPerRay + kSecondaryBytesPerRay; }

void carve_ray_queue(Carver& c, long cap, RayQueue* q) {
  q->ox = c.take<double>(cap); q->oy = c.take<double>(cap); q->oz = c.take<double>(cap);
  q->dx = c.take<double>(cap); q->dy = c.take<double>(cap); q->dz = c.take<double>(cap);
  q->t = c.take<double>(cap); q->w = c.take<double>(cap);
  q->rid = c.take<uint32_t>(cap); q->meta = c.take<uint32_t>(cap);
}

void carve_queues(Carver& c, long cap, RayQueue* q0, RayQueue* q1, SecondaryQueue* nq) {
  carve_ray_queue(c, cap, q0);
  carve_ray_queue(c, cap, q1);
  nq->rec = c.take<SecRec>(cap);
}

// Rays per chunk of the replay backward when the caller sizes the workspace
// with us_simulate_rf_vjp_workspace_size: about 160 bytes per ray and step
// plus 150 per ray, so some 20 GB for twelve interactions, and few enough
// chunks that the per-step launches stay long.
constexpr long kReplayChunk = 1L << 23;

// Vertex adjoints per copy, rounded up to 256 bytes.
long vadj_stride(const us_scene* scene) { return ((long)scene->mesh.n_vertices + 32) & ~31L; }

// Workspace of the replay backward for chunks of `cap` rays: dL/dh (and its
// f0 rows), the accumulators of the gradient, of the acquisition parameters
// and of the mesh vertex adjoints with the vertex totals, the step records,
// the queue of diffuse interactions with its step offsets, the per-step
// counts and the two live-ray queues.
struct ReplaySums {
  unsigned long long* g_sum = nullptr;
  unsigned long long* acq_sum = nullptr;
  unsigned long long* vadj = nullptr;
  double* vval = nullptr;
};

size_t replay_bytes(const us_scene* scene, int n_tx, const us_probe* p, int max_bounces, long cap,
                    ReplayStack* k = nullptr, char* base = nullptr, float** gh = nullptr,
                    float** gh_f0 = nullptr, ReplaySums* sums = nullptr, RayQueue* q0 = nullptr,
                    RayQueue* q1 = nullptr, unsigned long long** counts = nullptr,
                    uint32_t** sort_count = nullptr, uint32_t** sort_part = nullptr) {
  Carver c{base};
  float* g = c.take<float>((size_t)n_tx * p->d.n_elem * p->d.n_t);
  if (gh) *gh = g;
  float* gf = c.take<float>((size_t)n_tx * p->d.n_elem * p->d.n_t);
  if (gh_f0) *gh_f0 = gf;
  ReplaySums tmp_sums;
  ReplaySums& sm = sums ? *sums : tmp_sums;
  sm.g_sum = c.take<unsigned long long>((size_t)std::max(1, scene->q_offset) * kSumWords);
  sm.acq_sum = c.take<unsigned long long>((size_t)(n_tx + 3) * kSumWords);
  sm.vadj = c.take<unsigned long long>((size_t)kVadjCopies * vadj_stride(scene) * kSumWords);
  sm.vval = c.take<double>((size_t)vadj_stride(scene));
  ReplayStack tmp;
  ReplayStack& r = k ? *k : tmp;
  const size_t n = (size_t)cap * (max_bounces + 1);
  r.rec = c.take<StepRec>(n);
  r.adj = c.take<StepAdj>(n);
  r.last = c.take<int>((size_t)cap);
  r.queue = c.take<uint32_t>((size_t)cap * (max_bounces > 0 ? max_bounces : 1));
  r.queue_begin = c.take<unsigned long long>((size_t)max_bounces + 1);
  // receiver segments in key order (scenes with meshes and diffuse surfaces;
  // the per-step key counts are held to 2^26 words, else queue order)
  const bool sort = sorts_segments(scene) && (long)sort_keys(p) * std::max(1, max_bounces) <= (1L << 26);
  r.sort_kr = sort ? c.take<uint2>((size_t)cap * (max_bounces > 0 ? max_bounces : 1)) : nullptr;
  r.sort_q = sort ? c.take<uint32_t>((size_t)cap * (max_bounces > 0 ? max_bounces : 1)) : nullptr;
  uint32_t* sc = sort ? c.take<uint32_t>((size_t)sort_keys(p) * (max_bounces > 0 ? max_bounces : 1)) : nullptr;
  uint32_t* sp = sort ? c.take<uint32_t>((size_t)kSortBlocks) : nullptr;
  if (sort_count) *sort_count = sc;
  if (sort_part) *sort_part = sp;
  unsigned long long* cn = c.take<unsigned long long>((size_t)max_bounces + 2);
  if (counts) *counts = cn;
  RayQueue ta, tb;
  carve_ray_queue(c, cap, q0 ? q0 : &ta);
  carve_ray_queue(c, cap, q1 ? q1 : &tb);
  return c.off;
}

size_t queue_bytes(long cap) {
  Carver c{nullptr};
  RayQueue a, b;
  SecondaryQueue n;
  carve_queues(c, cap, &a, &b, &n);
  c.take<uint32_t>((size_t)kDepositsPerRay * cap);
  c.take<float2>((size_t)kDepositsPerRay * cap);
  return c.off;
}

int check_trace_args(const us_scene* scene, const us_probe* probe, const us_tx_desc* tx, int n_tx,
                     int rays_per_elem, int64_t ray_begin, int64_t ray_count, int max_bounces) {
  US_CHECK(scene && probe && tx, "simulate_rf: NULL scene, probe or tx");
  US_CHECK(scene->ctx == probe->ctx, "simulate_rf: scene and probe belong to different contexts");
  US_CHECK(n_tx >= 1, "simulate_rf: n_tx must be >= 1");
  US_CHECK(rays_per_elem >= 1, "simulate_rf: rays_per_elem must be >= 1");
  const int64_t total = (int64_t)probe->d.n_elem * rays_per_elem;
  US_CHECK(total < (int64_t(1) << 32), "simulate_rf: n_elem * rays_per_elem must be < 2^32");
  US_CHECK(ray_begin >= 0 && ray_count >= 0 && ray_begin + ray_count <= total,
           "simulate_rf: ray range outside [0, n_elem * rays_per_elem)");
  US_CHECK(max_bounces >= 0 && max_bounces <= 1000, "simulate_rf: max_bounces must be in [0, 1000]");
  for (int i = 0; i < n_tx; ++i)
    US_CHECK(std::fabs(tx[i].angle) < 0.5 * M_PI, "simulate_rf: steering angle must be in (-pi/2, pi/2)");
  return US_OK;
}

}  // namespace

extern "C" {

size_t us_simulate_rf_workspace_size(const us_scene* scene, const us_probe* probe, int32_t n_tx,
                                     int64_t ray_count, int32_t max_bounces) {
  if (!scene || !probe || n_tx < 1 || ray_count < 0 || max_bounces < 0) return 0;
  const int group = n_tx < kMaxTxPerLaunch ? n_tx : kMaxTxPerLaunch;
  long chunk = (long)std::min<int64_t>((int64_t)group * ray_count, kDefaultChunk);
  if (chunk < 256) chunk = 256;
  return trace_fixed_bytes(n_tx, probe, max_bounces, sorts_segments(scene)) + queue_bytes(chunk);
}

int us_simulate_rf(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_tx_desc* tx,
                   int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                   int64_t ray_count, int32_t max_bounces, float* rf_dev, int64_t* counters_dev,
                   uint64_t* ray_hash_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && rf_dev && ws_dev, "us_simulate_rf: NULL ctx, rf or workspace");
  int rc = check_trace_args(scene, probe, tx, n_tx, rays_per_elem, ray_begin, ray_count, max_bounces);
  if (rc) return rc;
  const bool sort = sorts_segments(scene);
  const size_t fixed = trace_fixed_bytes(n_tx, probe, max_bounces, sort);
  // largest chunk whose queues fit in the workspace
  long cap = 0;
  {
    long lo = 0, hi = (long)std::max<int64_t>(256, (int64_t)std::min(n_tx, kMaxTxPerLaunch) * ray_count);
    while (lo < hi) {
      const long mid = (lo + hi + 1) / 2;
      if (fixed + queue_bytes(mid) <= ws_bytes) lo = mid; else hi = mid - 1;
    }
    cap = lo;
  }
  if (cap < std::min<int64_t>(256, (int64_t)n_tx * ray_count) || (ray_count > 0 && cap < 1))
    return fail(US_ETOOBIG, "us_simulate_rf: workspace too small (see us_simulate_rf_workspace_size)");
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const us_probe_desc& pd = probe->d;
  Carver c{(char*)ws_dev};
  long long* h = c.take<long long>((size_t)n_tx * pd.n_elem * pd.n_t);
  // per-bounce counts, the deposit-shard counts, the histogram's overflow count
  unsigned long long* counts = c.take<unsigned long long>((size_t)max_bounces + 5 + kDepShards);
  const int rows = bin_rows(n_tx, probe);
  void* bin_scratch = rows > 0 ? (void*)c.take<char>(splat_scratch_bytes(rows)) : nullptr;
  TraceArgs a{};
  if (sort) {
    a.sort_count = c.take<uint32_t>((size_t)sort_keys(probe));
    a.sort_part = c.take<uint32_t>((size_t)kSortBlocks);
  }
  carve_queues(c, cap, &a.qin, &a.qout, &a.nee);
  const RayQueue q0 = a.qin, q1 = a.qout;
  // receiver segments marched in key order on mesh scenes (the walk is what
  // they spend their time on); the permutation lies over the interaction's
  // dead input queue
  if (sort) a.sort = seg_sort(probe);
  a.dep.key = c.take<uint32_t>((size_t)kDepositsPerRay * cap);
  a.dep.w = c.take<float2>((size_t)kDepositsPerRay * cap);
  a.dep_count = counts + max_bounces + 4;
  // the binned order (16-byte records: key, two tent weights) is written
  // over the first ray queue, which is dead by then (72 bytes per ray hold
  // the 2 x 16 bytes per ray)
  uint4* sorted = reinterpret_cast<uint4*>(q0.ox);
  US_CHECK((size_t)kDepositsPerRay * cap * sizeof(uint4) <=
               (size_t)(reinterpret_cast<char*>(q1.ox) - reinterpret_cast<char*>(q0.ox)),
           "us_simulate_rf: internal workspace layout");
  a.scene = scene_view(scene, probe);
  a.probe = probe->pv;
  a.seed = seed;
  a.rays_per_elem = rays_per_elem;
  a.max_bounces = max_bounces;
  a.ray_begin = ray_begin;
  a.ray_count = ray_count;
  a.counts = counts;
  a.h = h;
  a.hist_scale = hist_scale(rays_per_elem);
  a.hist_over = counts + max_bounces + 4 + kDepShards;
  a.counters = (unsigned long long*)counters_dev;
  a.hash = (unsigned long long*)ray_hash_dev;
  const bool audit = ray_hash_dev != nullptr;
  launch_fill_u32((uint32_t*)h, 2L * n_tx * pd.n_elem * pd.n_t, 0u, s);
  launch_fill_u32((uint32_t*)a.hist_over, 2, 0u, s);
  if (audit) launch_fill_u32((uint32_t*)ray_hash_dev, 2L * n_tx * ray_count, 0u, s);
  if (probe->M > kMaxTaps - 1) return fail(US_EINVAL, "us_simulate_rf: pulse too long");
  for (int t0 = 0; t0 < n_tx; t0 += kMaxTxPerLaunch) {
    const int ng = std::min(kMaxTxPerLaunch, n_tx - t0);
    fill_tx(a.tx, tx, t0, ng);
    a.tx_base = t0;
    const long total = (long)ng * ray_count;
    const int n_rows = ng * pd.n_elem;
    // deposits are binned (kDepShards shards of records) except on mesh scenes,
    // whose walk-bound secondary kernel hides global atomics into h
    a.dep_cap = (bin_scratch && n_rows <= rows && scene->n_meshes == 0) ? kDepositsPerRay * cap : 0;
    a.dep.row0 = (uint32_t)t0 * (uint32_t)pd.n_elem;
    bool filtered = false;   // the group's RF rows are written
    for (long g0 = 0; g0 < total; g0 += cap) {
      const long n = std::min(cap, total - g0);
      a.g0 = g0;
      a.n_chunk = n;
      launch_fill_u32((uint32_t*)counts, 2L * (max_bounces + 4 + kDepShards), 0u, s);
      a.qin = q0;
      a.qout = q1;
      for (int k = 1; k <= max_bounces + 1; ++k) {
        if (sort && k <= max_bounces) launch_fill_u32(a.sort_count, a.sort.keys, 0u, s);
        {
          Timed tm(ctx, "bounce", s);
          launch_bounce(a, k, n, audit, s);
        }
        if (k <= max_bounces && scene->any_diffuse) {
          if (sort) {
            a.sort_perm = reinterpret_cast<uint32_t*>(a.qin.ox);   // bounce k has consumed its input queue
            Timed tm(ctx, "secondary_sort", s);
            launch_secondary_sort(a, k, n, s);
          }
          Timed tm(ctx, "secondary", s);
          launch_secondary(a, k, n, audit, s);
        }
        std::swap(a.qin, a.qout);
      }
      if (a.dep_cap > 0) {
        {
          Timed tm(ctx, "splat_bin", s);
          launch_splat_bin(a.dep, a.dep_count, a.dep_cap / kDepShards, n_rows, sorted, bin_scratch, s);
        }
        // the group's last chunk: its deposits, the row of h and the pulse in
        // one pass; earlier chunks add their deposits to h
        if (g0 + n >= total) {
          Timed tm(ctx, "splat_pulse", s);
          filtered = launch_splat_pulse(sorted, bin_scratch, a.dep.row0, n_rows, pd.n_t, h, a.hist_scale,
                                        a.hist_over, probe->taps, probe->M, rf_dev, s) == 0;
        }
        if (!filtered) {
          Timed tm(ctx, "splat_accumulate", s);
          launch_splat_accumulate(sorted, bin_scratch, a.dep.row0, n_rows, pd.n_t, h, a.hist_scale, a.hist_over, s);
        }
      }
    }
    if (!filtered) {
      const long r0 = (long)t0 * pd.n_elem;
      Timed tm(ctx, "pulse", s);
      launch_pulse_fixed(h + r0 * pd.n_t, a.hist_scale, a.hist_over, rf_dev + r0 * pd.n_t, probe->taps, probe->M,
                         pd.n_t, n_rows, s);
    }
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

}  // extern "C"

namespace {

GridView grid_view(const us_grid_desc* g) {
  return GridView{g->n_x, g->n_z, g->x0, g->dx, g->z0, g->dz};
}

int check_beamform(const us_probe* probe, const us_grid_desc* grid, const us_tx_desc* tx, int n_tx) {
  US_CHECK(probe && grid && tx, "beamform: NULL probe, grid or tx");
  US_CHECK(n_tx >= 1, "beamform: n_tx must be >= 1");
  US_CHECK(probe->twiddle != nullptr && probe->d.n_t >= 64 && probe->d.n_t <= 8192,
           "beamform: n_t must be a power of two in [64, 8192]");
  US_CHECK(grid->n_x >= 1 && grid->n_z >= 1 && (int64_t)grid->n_x * grid->n_z < (int64_t(1) << 31),
           "beamform: grid size out of range");
  US_CHECK(grid->dx > 0 && grid->dz > 0 && grid->z0 >= 0, "beamform: need dx, dz > 0 and z0 >= 0");
  for (int i = 0; i < n_tx; ++i)
    US_CHECK(std::fabs(tx[i].angle) < 0.5 * M_PI, "beamform: steering angle must be in (-pi/2, pi/2)");
  return US_OK;
}

}  // namespace

extern "C" {

size_t us_beamform_workspace_size(const us_probe* probe, int32_t n_tx) {
  if (!probe || n_tx < 1) return 0;
  return align_up((size_t)n_tx * probe->d.n_elem * probe->d.n_t * sizeof(float2));
}

}  // extern "C"

namespace {

// The launches of us_beamform with the analytic signal in A (checked by the
// caller); `timed` brackets them with the profiling events when profiling is on.
int beamform_launch(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid, const us_tx_desc* tx,
                    int32_t n_tx, const float* rf_dev, float* iq_dev, float2* A, hipStream_t s, bool timed) {
  const long rows = (long)n_tx * probe->d.n_elem;
  {
    Timed tm(ctx, timed ? "analytic" : nullptr, s);
    if (launch_analytic(rf_dev, A, probe->twiddle, probe->d.n_t, rows, s))
      return fail(US_EINVAL, "us_beamform: unsupported n_t");
  }
  const GridView g = grid_view(grid);
  for (int t0 = 0; t0 < n_tx; t0 += kMaxTxPerLaunch) {
    const int ng = std::min(kMaxTxPerLaunch, n_tx - t0);
    TxTable tt;
    fill_tx(tt, tx, t0, ng);
    Timed tm(ctx, timed ? "das" : nullptr, s);
    launch_das(A, (float2*)iq_dev, probe->pv, g, tt, ng, t0, t0 > 0, s);
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

}  // namespace

extern "C" {

int us_beamform(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid, const us_tx_desc* tx,
                int32_t n_tx, const float* rf_dev, float* iq_dev, void* ws_dev, size_t ws_bytes,
                void* stream) {
  US_CHECK(ctx && rf_dev && iq_dev && ws_dev, "us_beamform: NULL argument");
  int rc = check_beamform(probe, grid, tx, n_tx);
  if (rc) return rc;
  if (ws_bytes < us_beamform_workspace_size(probe, n_tx))
    return fail(US_ETOOBIG, "us_beamform: workspace too small");
  US_HIP(bind_device(ctx->device));
  return beamform_launch(ctx, probe, grid, tx, n_tx, rf_dev, iq_dev, (float2*)ws_dev, (hipStream_t)stream, true);
}

int us_beamform_static(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid, const us_tx_desc* tx,
                       int32_t n_tx, const float* rf_dev, float* iq_dev, void* stream) {
  US_CHECK(ctx && rf_dev && iq_dev, "us_beamform_static: NULL argument");
  int rc = check_beamform(probe, grid, tx, n_tx);
  if (rc) return rc;
  const size_t need = us_beamform_workspace_size(probe, n_tx);
  if (need > kStaticScratchBytes)
    return fail(US_ETOOBIG, "us_beamform_static: the analytic signal needs " + std::to_string(need) +
                                " bytes; the static scratch holds " + std::to_string(kStaticScratchBytes) +
                                " (use us_beamform with a workspace)");
  void* p = ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
  US_CHECK(p != nullptr, "us_beamform_static: no static scratch on this device");
  US_HIP(bind_device(ctx->device));
  return beamform_launch(ctx, probe, grid, tx, n_tx, rf_dev, iq_dev, (float2*)p, (hipStream_t)stream, false);
}

size_t us_bmode_workspace_size(int64_t n_px) {
  (void)n_px;
  return 2 * kAlign;
}

int us_bmode(us_ctx* ctx, const float* iq_dev, int64_t n_px, float dr_db, float* bmode_dev,
             void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && iq_dev && bmode_dev && ws_dev, "us_bmode: NULL argument");
  US_CHECK(n_px >= 1 && n_px < (int64_t(1) << 32) - 1, "us_bmode: n_px out of range");
  US_CHECK(dr_db > 0, "us_bmode: dr_db must be positive");
  if (ws_bytes < us_bmode_workspace_size(n_px)) return fail(US_ETOOBIG, "us_bmode: workspace too small");
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* key = (unsigned long long*)ws_dev;
  launch_fill_u32((uint32_t*)key, 2, 0u, s);
  {
    Timed tm(ctx, "bmode", s);
    launch_env_max((const float2*)iq_dev, n_px, key, s);
    launch_bmode((const float2*)iq_dev, n_px, dr_db, key, bmode_dev, s);
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

int us_bmode_vjp(us_ctx* ctx, const float* iq_dev, const float* g_bmode_dev, int64_t n_px,
                 float dr_db, float* g_iq_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && iq_dev && g_bmode_dev && g_iq_dev && ws_dev, "us_bmode_vjp: NULL argument");
  US_CHECK(n_px >= 1 && n_px < (int64_t(1) << 32) - 1, "us_bmode_vjp: n_px out of range");
  US_CHECK(dr_db > 0, "us_bmode_vjp: dr_db must be positive");
  if (ws_bytes < us_bmode_workspace_size(n_px)) return fail(US_ETOOBIG, "us_bmode_vjp: workspace too small");
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* key = (unsigned long long*)ws_dev;
  unsigned long long* sum = (unsigned long long*)((char*)ws_dev + kAlign);
  static_assert(kSumWords * 8 <= kAlign, "bmode workspace layout");
  launch_fill_u32((uint32_t*)key, 2, 0u, s);
  launch_fill_u32((uint32_t*)sum, 2 * kSumWords, 0u, s);
  {
    Timed tm(ctx, "bmode_vjp", s);
    launch_env_max((const float2*)iq_dev, n_px, key, s);
    launch_bmode_vjp((const float2*)iq_dev, g_bmode_dev, n_px, dr_db, key, sum, (float2*)g_iq_dev, s);
    launch_bmode_vjp_fix((const float2*)iq_dev, n_px, key, sum, (float2*)g_iq_dev, s);
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

size_t us_image_loss_workspace_size(int64_t n_px) {
  (void)n_px;
  return kAlign;
}

int us_image_loss(us_ctx* ctx, const float* bmode_dev, const float* ref_dev, int64_t n_px,
                  double lambda1, double lambda2, double* loss_dev, float* g_bmode_dev,
                  void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && bmode_dev && ref_dev && loss_dev && ws_dev, "us_image_loss: NULL argument");
  if (ws_bytes < us_image_loss_workspace_size(n_px)) return fail(US_ETOOBIG, "us_image_loss: workspace too small");
  US_CHECK(n_px >= 1, "us_image_loss: n_px must be >= 1");
  US_CHECK(lambda1 >= 0 && lambda2 >= 0, "us_image_loss: weights must be non-negative");
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  Timed tm(ctx, "image_loss", s);
  unsigned long long* acc = (unsigned long long*)ws_dev;
  static_assert(kSumWords * 8 <= kAlign, "loss workspace layout");
  launch_fill_u32((uint32_t*)acc, 2 * kSumWords, 0u, s);
  launch_image_loss(bmode_dev, ref_dev, n_px, lambda1, lambda2, acc, loss_dev, g_bmode_dev, s);
  US_HIP(hipGetLastError());
  return US_OK;
}

size_t us_beamform_vjp_workspace_size(const us_probe* probe, int32_t n_tx) {
  return us_beamform_workspace_size(probe, n_tx);
}

int us_beamform_vjp(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid,
                    const us_tx_desc* tx, int32_t n_tx, const float* g_iq_dev, float* g_rf_dev,
                    void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && g_iq_dev && g_rf_dev && ws_dev, "us_beamform_vjp: NULL argument");
  int rc = check_beamform(probe, grid, tx, n_tx);
  if (rc) return rc;
  if (ws_bytes < us_beamform_vjp_workspace_size(probe, n_tx))
    return fail(US_ETOOBIG, "us_beamform_vjp: workspace too small");
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  float2* gA = (float2*)ws_dev;
  const GridView g = grid_view(grid);
  for (int t0 = 0; t0 < n_tx; t0 += kMaxTxPerLaunch) {
    const int ng = std::min(kMaxTxPerLaunch, n_tx - t0);
    TxTable tt;
    fill_tx(tt, tx, t0, ng);
    Timed tm(ctx, "das_adjoint", s);
    launch_das_adjoint((const float2*)g_iq_dev, gA, probe->pv, g, tt, ng, t0, s);
  }
  {
    Timed tm(ctx, "analytic_adjoint", s);
    if (launch_analytic_adjoint(gA, g_rf_dev, probe->twiddle, probe->d.n_t,
                                (long)n_tx * probe->d.n_elem, s))
      return fail(US_EINVAL, "us_beamform_vjp: unsupported n_t");
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

size_t us_beamform_acq_vjp_workspace_size(const us_probe* probe, const us_grid_desc* grid, int32_t n_tx) {
  if (!probe || !grid || n_tx < 1 || grid->n_x < 1 || grid->n_z < 1) return 0;
  const long tiles = das_acq_tiles(grid_view(grid));
  return us_beamform_workspace_size(probe, n_tx) +
         align_up((size_t)std::min(n_tx, kMaxTxPerLaunch) * tiles * 3 * sizeof(double));
}

int us_beamform_acq_vjp(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid, const us_tx_desc* tx,
                        int32_t n_tx, const float* rf_dev, const float* g_iq_dev, double* g_acq_dev,
                        void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && rf_dev && g_iq_dev && g_acq_dev && ws_dev, "us_beamform_acq_vjp: NULL argument");
  int rc = check_beamform(probe, grid, tx, n_tx);
  if (rc) return rc;
  if (ws_bytes < us_beamform_acq_vjp_workspace_size(probe, grid, n_tx))
    return fail(US_ETOOBIG, "us_beamform_acq_vjp: workspace too small");
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  float2* A = (float2*)ws_dev;
  double* part = (double*)((char*)ws_dev + us_beamform_workspace_size(probe, n_tx));
  const long rows = (long)n_tx * probe->d.n_elem;
  {
    Timed tm(ctx, "analytic", s);
    if (launch_analytic(rf_dev, A, probe->twiddle, probe->d.n_t, rows, s))
      return fail(US_EINVAL, "us_beamform_acq_vjp: unsupported n_t");
  }
  launch_fill_u32((uint32_t*)g_acq_dev, 2L * (n_tx + 2), 0u, s);
  const GridView g = grid_view(grid);
  for (int t0 = 0; t0 < n_tx; t0 += kMaxTxPerLaunch) {
    const int ng = std::min(kMaxTxPerLaunch, n_tx - t0);
    TxTable tt;
    fill_tx(tt, tx, t0, ng);
    Timed tm(ctx, "das_acq", s);
    launch_das_acq(A, (const float2*)g_iq_dev, probe->pv, g, tt, ng, t0, n_tx, part, g_acq_dev, s);
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

size_t us_simulate_rf_vjp_workspace_size(const us_scene* scene, const us_probe* probe,
                                         int32_t n_tx, int64_t ray_count, int32_t max_bounces) {
  if (!scene || !probe || n_tx < 1 || ray_count < 0 || max_bounces < 0) return 0;
  const int group = n_tx < kMaxTxPerLaunch ? n_tx : kMaxTxPerLaunch;
  const long cap = std::max(1L, std::min((long)group * (long)ray_count, kReplayChunk));
  return replay_bytes(scene, n_tx, probe, max_bounces, cap);
}

}  // extern "C"

namespace {

// The replay backward; g_acq_dev (may be null) also receives the adjoints of
// the acquisition parameters. The gradient arrives as dL/drf (g_rf_dev), or,
// with g_A_dev instead, as the gradient of the analytic signal, taken through
// the analytic map's and the pulse's adjoints in one kernel (no g_acq then).
// Workspace of a recorded frame (one transmit group, one chunk holding all
// n_tx * ray_count rays): the replay's, then the deposit histogram and its
// overflow count, then the march records of the first kMarchPerRay * rays
// queued diffuse interactions.
struct RecordedLayout {
  size_t replay = 0, total = 0;
  long long* h = nullptr;
  unsigned long long* over = nullptr;
  MarchRecs march{};
};
RecordedLayout recorded_layout(const us_scene* scene, const us_probe* p, int n_tx, int64_t ray_count,
                               int max_bounces, char* base) {
  RecordedLayout L;
  const long cap = (long)n_tx * ray_count;
  L.replay = replay_bytes(scene, n_tx, p, max_bounces, cap);
  size_t off = align_up(L.replay);
  const size_t hbytes = (size_t)n_tx * p->d.n_elem * p->d.n_t * sizeof(long long);
  if (base) L.h = (long long*)(base + off);
  off += align_up(hbytes);
  if (base) L.over = (unsigned long long*)(base + off);
  off += kAlign;
  const long mc = max_bounces > 0 && scene->any_diffuse ? kMarchPerRay * cap : 0;
  auto carve = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  if (mc) {
    L.march.cap = base ? mc : 0;
    L.march.tof = (double*)carve((size_t)mc * sizeof(double));
    L.march.att = (double*)carve((size_t)mc * sizeof(double));
    L.march.trans = (double*)carve((size_t)mc * sizeof(double));
    L.march.nstate = (uint32_t*)carve((size_t)mc * sizeof(uint32_t));
    L.march.s = (double*)carve((size_t)mc * kMarchLegs * sizeof(double));
    L.march.h = (int*)carve((size_t)mc * kMarchLegs * sizeof(int));
  }
  L.total = off;
  return L;
}
size_t recorded_bytes(const us_scene* scene, const us_probe* p, int n_tx, int64_t ray_count, int max_bounces) {
  return recorded_layout(scene, p, n_tx, ray_count, max_bounces, nullptr).total;
}

// FNV-1a over the transmit table, to tell a recorded frame's transmits apart.
uint64_t tx_hash(const us_tx_desc* tx, int n_tx) {
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(tx);
  for (size_t i = 0; i < (size_t)n_tx * sizeof(us_tx_desc); ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

int check_recorded_shape(const us_scene* scene, const us_probe* probe, int n_tx, int64_t ray_count,
                         int max_bounces, size_t ws_bytes) {
  US_CHECK(n_tx <= kMaxTxPerLaunch, "recorded frame: at most 64 transmits (one launch group)");
  US_CHECK(ray_count >= 1, "recorded frame: ray_count must be >= 1");
  if (ws_bytes < recorded_bytes(scene, probe, n_tx, ray_count, max_bounces))
    return fail(US_ETOOBIG, "recorded frame: workspace too small (see us_recorded_workspace_size)");
  return US_OK;
}

int check_recorded(const us_scene* scene, const us_probe* probe, const us_tx_desc* tx, int n_tx, uint64_t seed,
                   int rays_per_elem, int64_t ray_begin, int64_t ray_count, int max_bounces, const void* ws,
                   size_t ws_bytes) {
  const int rc = check_recorded_shape(scene, probe, n_tx, ray_count, max_bounces, ws_bytes);
  if (rc) return rc;
  const auto& r = scene->rec;
  US_CHECK(r.ws == ws && r.version == scene->version && r.probe == probe && r.seed == seed &&
               r.tx_hash == tx_hash(tx, n_tx) && r.ray_begin == ray_begin && r.ray_count == ray_count &&
               r.rays_per_elem == rays_per_elem && r.max_bounces == max_bounces && r.n_tx == n_tx,
           "recorded backward: the workspace holds no recorded forward of these arguments and parameters");
  return US_OK;
}

int simulate_rf_vjp(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_tx_desc* tx,
                    int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin, int64_t ray_count,
                    int32_t max_bounces, const float* g_rf_dev, double* g_theta_dev, double* g_acq_dev,
                    void* ws_dev, size_t ws_bytes, void* stream, const float2* g_A_dev = nullptr,
                    bool recorded = false) {
  US_CHECK(ctx && (g_rf_dev || g_A_dev) && g_theta_dev && ws_dev, "us_simulate_rf_vjp: NULL argument");
  US_CHECK(!(g_A_dev && g_acq_dev), "us_simulate_rf_vjp: acquisition gradients need dL/drf");
  int rc = check_trace_args(scene, probe, tx, n_tx, rays_per_elem, ray_begin, ray_count, max_bounces);
  if (rc) return rc;
  long cap = 0;
  if (recorded) {
    // the records of the whole frame, one chunk, from us_simulate_rf_recorded
    rc = check_recorded(scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces,
                        ws_dev, ws_bytes);
    if (rc) return rc;
    cap = (long)n_tx * ray_count;
  } else {
    // largest chunk that fits the workspace
    if (replay_bytes(scene, n_tx, probe, max_bounces, 1) > ws_bytes)
      return fail(US_ETOOBIG, "us_simulate_rf_vjp: workspace too small");
    long lo = 1, hi = kReplayChunk;
    while (lo < hi) {
      const long mid = lo + (hi - lo + 1) / 2;
      if (replay_bytes(scene, n_tx, probe, max_bounces, mid) <= ws_bytes) lo = mid; else hi = mid - 1;
    }
    cap = lo;
  }
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const us_probe_desc& pd = probe->d;
  ReplayArgs a{};
  float* gh = nullptr;
  float* gh_f0 = nullptr;
  RayQueue q0, q1;
  ReplaySums sums;
  replay_bytes(scene, n_tx, probe, max_bounces, cap, &a.stk, (char*)ws_dev, &gh, &gh_f0, &sums, &q0, &q1,
               &a.counts, &a.sort_count, &a.sort_part);
  if (a.sort_count) a.sort = seg_sort(probe);
  if (recorded) {   // the marches the recorded forward made
    const RecordedLayout lay = recorded_layout(scene, probe, n_tx, ray_count, max_bounces, (char*)ws_dev);
    a.march = lay.march;
  }
  a.vadj = sums.vadj;
  a.g_sum = sums.g_sum;
  a.acq_sum = sums.acq_sum;
  a.vadj_stride = vadj_stride(scene);
  if (scene->n_meshes > 0) launch_fill_u32((uint32_t*)a.vadj, 2L * kVadjCopies * a.vadj_stride * kSumWords, 0u, s);
  launch_fill_u32((uint32_t*)a.g_sum, 2L * std::max(1, scene->q_offset) * kSumWords, 0u, s);
  if (g_acq_dev) launch_fill_u32((uint32_t*)a.acq_sum, 2L * (n_tx + 3) * kSumWords, 0u, s);
  if (g_A_dev) {
    Timed tm(ctx, "analytic_pulse_adjoint", s);
    if (launch_analytic_pulse_adjoint(g_A_dev, gh, probe->twiddle, probe->taps_rev, probe->M, pd.n_t,
                                      (long)n_tx * pd.n_elem, s))
      return fail(US_EINVAL, "us_frame_vjp: unsupported n_t or pulse too long");
  } else {
    Timed tm(ctx, "pulse_adjoint", s);
    if (launch_pulse_adjoint(g_rf_dev, gh, probe->taps_rev, probe->M, pd.n_t, (long)n_tx * pd.n_elem, s))
      return fail(US_EINVAL, "us_simulate_rf_vjp: pulse too long");
    // with g_acq, also the rows of dL/dh for the pulse's derivative in f0
    if (g_acq_dev &&
        launch_pulse_adjoint(g_rf_dev, gh_f0, probe->dtaps_rev, probe->M, pd.n_t, (long)n_tx * pd.n_elem, s))
      return fail(US_EINVAL, "us_simulate_rf_vjp: pulse too long");
  }
  a.scene = scene_view(scene, probe);
  a.probe = probe->pv;
  a.seed = seed;
  a.rays_per_elem = rays_per_elem;
  a.max_bounces = max_bounces;
  a.ray_begin = ray_begin;
  a.ray_count = ray_count;
  a.n_params = scene->n_params;
  a.n_grad = scene->q_offset;
  a.grad_copies = 1;   // each launcher sets the copies its kernel's LDS allows
  a.gh = gh;
  a.cap = cap;
  a.g_acq = g_acq_dev;
  a.gh_f0 = g_acq_dev ? gh_f0 : nullptr;
  a.n_tx_total = n_tx;
  for (int t0 = 0; t0 < n_tx && ray_count > 0; t0 += kMaxTxPerLaunch) {
    const int ng = std::min(kMaxTxPerLaunch, n_tx - t0);
    fill_tx(a.tx, tx, t0, ng);
    a.tx_base = t0;
    const long n_group = (long)ng * ray_count;
    for (long g0 = 0; g0 < n_group; g0 += cap) {
      const long n = std::min(cap, n_group - g0);
      a.g0 = g0;
      if (!recorded) {   // a recorded forward left the records, the queue and its order
        launch_fill_u32((uint32_t*)a.counts, 2L * (max_bounces + 2), 0u, s);
        if (a.sort.keys > 0) launch_fill_u32(a.sort_count, (long)a.sort.keys * max_bounces, 0u, s);
        Timed tm(ctx, "replay_forward", s);
        for (int k = 1; k <= max_bounces + 1; ++k) {
          a.qout = (k & 1) ? q0 : q1;
          a.qin = (k & 1) ? q1 : q0;
          launch_replay_forward(a, k, n, s);
        }
      }
      {
        Timed tm(ctx, "replay_secondary", s);
        if (!recorded) {
          launch_replay_prefix(a, s);
          launch_replay_sort(a, n * std::max(1, max_bounces), s);
        }
        launch_replay_secondary(a, n * std::max(1, max_bounces), s);
      }
      {
        Timed tm(ctx, "replay_reverse", s);
        launch_replay_reverse(a, n, s);
      }
    }
  }
  // f0 also scales every region's amplitude attenuation a_r = alpha_r np_per_m,
  // so the f0 entry takes sum_r alpha_r dL/dalpha_r / f0 besides
  launch_grad_finish(a.g_sum, a.n_grad, g_theta_dev, a.acq_sum, n_tx + 3, g_acq_dev, n_tx + 2, a.scene.theta,
                     scene->n_regions, 1.0 / pd.f0, s);
  if (scene->n_meshes > 0) {
    Timed tm(ctx, "basis_gather", s);
    launch_basis_gather(a.vadj, a.vadj_stride, scene->mesh.n_vertices, sums.vval, scene->mesh.vbasis,
                        scene->mesh.vbeg, scene->n_meshes, scene->n_basis, g_theta_dev + scene->q_offset, s);
  }
  US_HIP(hipGetLastError());
  return US_OK;
}

}  // namespace

extern "C" {

int us_simulate_rf_vjp(us_ctx* ctx, const us_scene* scene, const us_probe* probe,
                       const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                       int64_t ray_begin, int64_t ray_count, int32_t max_bounces,
                       const float* g_rf_dev, double* g_theta_dev, void* ws_dev, size_t ws_bytes,
                       void* stream) {
  return simulate_rf_vjp(ctx, scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces,
                         g_rf_dev, g_theta_dev, nullptr, ws_dev, ws_bytes, stream);
}

int us_simulate_rf_vjp_acq(us_ctx* ctx, const us_scene* scene, const us_probe* probe,
                           const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                           int64_t ray_begin, int64_t ray_count, int32_t max_bounces,
                           const float* g_rf_dev, double* g_theta_dev, double* g_acq_dev, void* ws_dev,
                           size_t ws_bytes, void* stream) {
  US_CHECK(g_acq_dev, "us_simulate_rf_vjp_acq: NULL g_acq");
  return simulate_rf_vjp(ctx, scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces,
                         g_rf_dev, g_theta_dev, g_acq_dev, ws_dev, ws_bytes, stream);
}

// Workspace of us_frame_vjp: the B-mode adjoint's frame maximum and sum, the
// image gradient, the analytic-signal gradient and the replay's workspace.
size_t us_frame_vjp_workspace_size(const us_scene* scene, const us_probe* probe, const us_grid_desc* grid,
                                   int32_t n_tx, int64_t ray_count, int32_t max_bounces) {
  if (!scene || !probe || !grid || n_tx < 1 || grid->n_x < 1 || grid->n_z < 1) return 0;
  const size_t replay = us_simulate_rf_vjp_workspace_size(scene, probe, n_tx, ray_count, max_bounces);
  if (!replay) return 0;
  const int64_t n_px = (int64_t)grid->n_x * grid->n_z;
  return us_bmode_workspace_size(n_px) + align_up((size_t)n_px * sizeof(float2)) +
         us_beamform_workspace_size(probe, n_tx) + replay;
}

}  // extern "C"

namespace {

// The image half of the frame backward: dL/dB to dL/dA in gA (carved from w
// after the B-mode sums and dL/dI); returns the first byte after gA.
char* frame_image_vjp(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid, const us_tx_desc* tx,
                      int32_t n_tx, const float* iq_dev, const float* g_bmode_dev, float dr_db, char* w,
                      float2** gA_out, hipStream_t s) {
  const int64_t n_px = (int64_t)grid->n_x * grid->n_z;
  unsigned long long* key = (unsigned long long*)w;
  unsigned long long* sum = (unsigned long long*)(w + kAlign);
  w += us_bmode_workspace_size(n_px);
  float2* g_iq = (float2*)w;
  w += align_up((size_t)n_px * sizeof(float2));
  float2* gA = (float2*)w;
  w += us_beamform_workspace_size(probe, n_tx);
  launch_fill_u32((uint32_t*)key, 2, 0u, s);
  launch_fill_u32((uint32_t*)sum, 2 * kSumWords, 0u, s);
  {
    Timed tm(ctx, "bmode_vjp", s);
    launch_env_max((const float2*)iq_dev, n_px, key, s);
    launch_bmode_vjp((const float2*)iq_dev, g_bmode_dev, n_px, dr_db, key, sum, g_iq, s);
    launch_bmode_vjp_fix((const float2*)iq_dev, n_px, key, sum, g_iq, s);
  }
  const GridView g = grid_view(grid);
  for (int t0 = 0; t0 < n_tx; t0 += kMaxTxPerLaunch) {
    const int ng = std::min(kMaxTxPerLaunch, n_tx - t0);
    TxTable tt;
    fill_tx(tt, tx, t0, ng);
    Timed tm(ctx, "das_adjoint", s);
    launch_das_adjoint(g_iq, gA, probe->pv, g, tt, ng, t0, s);
  }
  *gA_out = gA;
  return w;
}

size_t frame_image_bytes(const us_probe* probe, const us_grid_desc* grid, int32_t n_tx) {
  const int64_t n_px = (int64_t)grid->n_x * grid->n_z;
  return us_bmode_workspace_size(n_px) + align_up((size_t)n_px * sizeof(float2)) +
         us_beamform_workspace_size(probe, n_tx);
}

}  // namespace

extern "C" {

int us_frame_vjp(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_grid_desc* grid,
                 const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                 int64_t ray_count, int32_t max_bounces, const float* iq_dev, const float* g_bmode_dev,
                 float dr_db, double* g_theta_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && iq_dev && g_bmode_dev && g_theta_dev && ws_dev, "us_frame_vjp: NULL argument");
  US_CHECK(dr_db > 0, "us_frame_vjp: dr_db must be positive");
  int rc = check_beamform(probe, grid, tx, n_tx);
  if (rc) return rc;
  rc = check_trace_args(scene, probe, tx, n_tx, rays_per_elem, ray_begin, ray_count, max_bounces);
  if (rc) return rc;
  // the image buffers and the replay of chunks of one ray at least, as us_simulate_rf_vjp
  if (ws_bytes < frame_image_bytes(probe, grid, n_tx) + replay_bytes(scene, n_tx, probe, max_bounces, 1))
    return fail(US_ETOOBIG, "us_frame_vjp: workspace too small");
  US_HIP(bind_device(ctx->device));
  float2* gA = nullptr;
  char* w = frame_image_vjp(ctx, probe, grid, tx, n_tx, iq_dev, g_bmode_dev, dr_db, (char*)ws_dev, &gA,
                            (hipStream_t)stream);
  return simulate_rf_vjp(ctx, scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces,
                         nullptr, g_theta_dev, nullptr, w, ws_bytes - (size_t)(w - (char*)ws_dev), stream, gA);
}

size_t us_recorded_workspace_size(const us_scene* scene, const us_probe* probe, int32_t n_tx, int64_t ray_count,
                                  int32_t max_bounces) {
  if (!scene || !probe || n_tx < 1 || n_tx > kMaxTxPerLaunch || ray_count < 1 || max_bounces < 0) return 0;
  return recorded_bytes(scene, probe, n_tx, ray_count, max_bounces);
}

int us_simulate_rf_recorded(us_ctx* ctx, us_scene* scene, const us_probe* probe, const us_tx_desc* tx,
                            int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                            int64_t ray_count, int32_t max_bounces, float* rf_dev, int64_t* counters_dev,
                            void* ws_dev, size_t ws_bytes, void* stream) {
  US_CHECK(ctx && rf_dev && ws_dev, "us_simulate_rf_recorded: NULL ctx, rf or workspace");
  int rc = check_trace_args(scene, probe, tx, n_tx, rays_per_elem, ray_begin, ray_count, max_bounces);
  if (rc) return rc;
  rc = check_recorded_shape(scene, probe, n_tx, ray_count, max_bounces, ws_bytes);
  if (rc) return rc;
  if (probe->M > kMaxTaps - 1) return fail(US_EINVAL, "us_simulate_rf_recorded: pulse too long");
  scene->rec.ws = nullptr;   // valid again only once this call has been queued whole
  US_HIP(bind_device(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const us_probe_desc& pd = probe->d;
  const long cap = (long)n_tx * ray_count;
  ReplayArgs a{};
  float* gh = nullptr;
  float* gh_f0 = nullptr;
  RayQueue q0, q1;
  ReplaySums sums;
  const size_t rb = replay_bytes(scene, n_tx, probe, max_bounces, cap, &a.stk, (char*)ws_dev, &gh, &gh_f0, &sums,
                                 &q0, &q1, &a.counts, &a.sort_count, &a.sort_part);
  if (a.sort_count) a.sort = seg_sort(probe);
  (void)rb;
  const RecordedLayout lay = recorded_layout(scene, probe, n_tx, ray_count, max_bounces, (char*)ws_dev);
  const long rows = (long)n_tx * pd.n_elem;
  a.h = lay.h;
  a.hist_over = lay.over;
  a.hist_scale = hist_scale(rays_per_elem);
  a.march = lay.march;
  a.counters = (unsigned long long*)counters_dev;
  launch_fill_u32((uint32_t*)a.h, 2L * rows * pd.n_t, 0u, s);
  launch_fill_u32((uint32_t*)a.hist_over, 2, 0u, s);
  launch_fill_u32((uint32_t*)a.counts, 2L * (max_bounces + 2), 0u, s);
  if (a.sort.keys > 0) launch_fill_u32(a.sort_count, (long)a.sort.keys * max_bounces, 0u, s);
  a.scene = scene_view(scene, probe);
  a.probe = probe->pv;
  a.seed = seed;
  a.rays_per_elem = rays_per_elem;
  a.max_bounces = max_bounces;
  a.ray_begin = ray_begin;
  a.ray_count = ray_count;
  a.n_params = scene->n_params;
  a.n_grad = scene->q_offset;
  a.grad_copies = 1;
  a.cap = cap;
  a.n_tx_total = n_tx;
  fill_tx(a.tx, tx, 0, n_tx);
  a.tx_base = 0;
  a.g0 = 0;
  {
    Timed tm(ctx, "recorded_forward", s);
    for (int k = 1; k <= max_bounces + 1; ++k) {
      a.qout = (k & 1) ? q0 : q1;
      a.qin = (k & 1) ? q1 : q0;
      launch_replay_forward(a, k, cap, s);
    }
  }
  {
    Timed tm(ctx, "recorded_deposit", s);
    launch_replay_prefix(a, s);
    launch_replay_sort(a, cap * std::max(1, max_bounces), s);
    if (max_bounces > 0 && scene->any_diffuse) launch_replay_deposit(a, cap * std::max(1, max_bounces), s);
  }
  {
    Timed tm(ctx, "pulse", s);
    launch_pulse_fixed(a.h, a.hist_scale, a.hist_over, rf_dev, probe->taps, probe->M, pd.n_t, (int)rows, s);
  }
  US_HIP(hipGetLastError());
  scene->rec.ws = ws_dev;
  scene->rec.version = scene->version;
  scene->rec.probe = probe;
  scene->rec.seed = seed;
  scene->rec.tx_hash = tx_hash(tx, n_tx);
  scene->rec.ray_begin = ray_begin;
  scene->rec.ray_count = ray_count;
  scene->rec.rays_per_elem = rays_per_elem;
  scene->rec.max_bounces = max_bounces;
  scene->rec.n_tx = n_tx;
  return US_OK;
}

int us_simulate_rf_vjp_recorded(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_tx_desc* tx,
                                int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                                int64_t ray_count, int32_t max_bounces, const float* g_rf_dev, double* g_theta_dev,
                                void* ws_dev, size_t ws_bytes, void* stream) {
  return simulate_rf_vjp(ctx, scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces,
                         g_rf_dev, g_theta_dev, nullptr, ws_dev, ws_bytes, stream, nullptr, true);
}

size_t us_frame_vjp_recorded_workspace_size(const us_probe* probe, const us_grid_desc* grid, int32_t n_tx) {
  if (!probe || !grid || n_tx < 1 || grid->n_x < 1 || grid->n_z < 1) return 0;
  return frame_image_bytes(probe, grid, n_tx);
}

int us_frame_vjp_recorded(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_grid_desc* grid,
                          const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                          int64_t ray_begin, int64_t ray_count, int32_t max_bounces, const float* iq_dev,
                          const float* g_bmode_dev, float dr_db, double* g_theta_dev, void* ws_dev,
                          size_t ws_bytes, void* rec_dev, size_t rec_bytes, void* stream) {
  US_CHECK(ctx && iq_dev && g_bmode_dev && g_theta_dev && ws_dev && rec_dev, "us_frame_vjp_recorded: NULL argument");
  US_CHECK(dr_db > 0, "us_frame_vjp_recorded: dr_db must be positive");
  int rc = check_beamform(probe, grid, tx, n_tx);
  if (rc) return rc;
  rc = check_trace_args(scene, probe, tx, n_tx, rays_per_elem, ray_begin, ray_count, max_bounces);
  if (rc) return rc;
  if (ws_bytes < frame_image_bytes(probe, grid, n_tx))
    return fail(US_ETOOBIG, "us_frame_vjp_recorded: workspace too small");
  rc = check_recorded(scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces, rec_dev,
                      rec_bytes);
  if (rc) return rc;
  US_HIP(bind_device(ctx->device));
  float2* gA = nullptr;
  frame_image_vjp(ctx, probe, grid, tx, n_tx, iq_dev, g_bmode_dev, dr_db, (char*)ws_dev, &gA, (hipStream_t)stream);
  return simulate_rf_vjp(ctx, scene, probe, tx, n_tx, seed, rays_per_elem, ray_begin, ray_count, max_bounces,
                         nullptr, g_theta_dev, nullptr, rec_dev, rec_bytes, stream, gA, true);
}

int us_param_map(us_ctx* ctx, const double* u_dev, const double* lo_dev, const double* hi_dev,
                 int32_t n, double* theta_dev, void* stream) {
  US_CHECK(ctx && u_dev && lo_dev && hi_dev && theta_dev, "us_param_map: NULL argument");
  US_CHECK(n >= 1, "us_param_map: n must be >= 1");
  US_HIP(bind_device(ctx->device));
  Timed tm(ctx, "param_map", (hipStream_t)stream);
  launch_param_map(u_dev, lo_dev, hi_dev, n, theta_dev, (hipStream_t)stream);
  US_HIP(hipGetLastError());
  return US_OK;
}

int us_adam_step(us_ctx* ctx, double* u_dev, double* m_dev, double* v_dev,
                 const double* g_theta_dev, const double* lo_dev, const double* hi_dev,
                 const double* lr_dev, int32_t n, int32_t step, double beta1, double beta2,
                 double eps, double max_norm, void* stream) {
  US_CHECK(ctx && u_dev && m_dev && v_dev && g_theta_dev && lo_dev && hi_dev && lr_dev,
           "us_adam_step: NULL argument");
  US_CHECK(n >= 1, "us_adam_step: n must be >= 1");
  US_CHECK(step >= 1, "us_adam_step: step counts from 1");
  US_CHECK(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0,
           "us_adam_step: need 0 <= beta1, beta2 < 1 and eps > 0");
  US_HIP(bind_device(ctx->device));
  Timed tm(ctx, "adam_step", (hipStream_t)stream);
  launch_adam(u_dev, m_dev, v_dev, g_theta_dev, lo_dev, hi_dev, lr_dev, n, step, beta1, beta2, eps,
              max_norm, (hipStream_t)stream);
  US_HIP(hipGetLastError());
  return US_OK;
}

int us_profile_enable(us_ctx* ctx, int enable) {
  US_CHECK(ctx, "us_profile_enable: NULL ctx");
  ctx->prof.on = enable != 0;
  return US_OK;
}

int us_profile_read(us_ctx* ctx, int32_t max_kernels, char* names, double* total_ms,
                    int64_t* launches, int32_t* n_kernels) {
  US_CHECK(ctx && n_kernels && (max_kernels == 0 || (names && total_ms && launches)),
           "us_profile_read: NULL argument");
  US_HIP(bind_device(ctx->device));
  ProfileLog& L = ctx->prof;
  for (auto& p : L.pending) {
    US_HIP(hipEventSynchronize(p.b));
    float ms = 0.0f;
    US_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    bool found = false;
    for (auto& t : L.totals)
      if (t.first == p.name) { t.second.first += ms; t.second.second += 1; found = true; }
    if (!found) L.totals.push_back({p.name, {ms, 1}});
    L.pool.push_back(p.a);
    L.pool.push_back(p.b);
  }
  L.pending.clear();
  int n = 0;
  for (auto& t : L.totals) {
    if (n >= max_kernels) break;
    std::strncpy(names + 32 * n, t.first.c_str(), 31);
    names[32 * n + 31] = 0;
    total_ms[n] = t.second.first;
    launches[n] = t.second.second;
    ++n;
  }
  *n_kernels = n;
  L.totals.clear();
  return US_OK;
}

}  // extern "C"
