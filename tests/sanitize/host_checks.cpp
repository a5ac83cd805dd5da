// Host-side checks of the library built with AddressSanitizer and
// UndefinedBehaviorSanitizer (no GPU needed): the hierarchy builder on closed
// meshes and on degenerate input, the order-independent sums' windows, and
// the argument checks of the C-ABI entry points. Exits non-zero on a failed
// check; the sanitizers abort on the first report.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "kernels.h"
#include "usrt.h"

using namespace usrt;

static int g_fail = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) { std::printf("FAILED %s:%d %s\n", __FILE__, __LINE__, #c); ++g_fail; } \
  } while (0)

// A UV sphere of radius r about c: n_lat x n_lon quads as triangles, poles fanned.
static void uv_sphere(double cx, double cy, double cz, double r, int n_lat, int n_lon, int mesh,
                      std::vector<double>& v, std::vector<int32_t>& t, std::vector<int32_t>& tm) {
  const int base = (int)(v.size() / 3);
  v.insert(v.end(), {cx, cy, cz + r});
  for (int i = 1; i < n_lat; ++i)
    for (int j = 0; j < n_lon; ++j) {
      const double th = M_PI * i / n_lat, ph = 2 * M_PI * j / n_lon;
      v.insert(v.end(), {cx + r * std::sin(th) * std::cos(ph), cy + r * std::sin(th) * std::sin(ph),
                         cz + r * std::cos(th)});
    }
  v.insert(v.end(), {cx, cy, cz - r});
  const int south = (int)(v.size() / 3) - 1;
  auto ring = [&](int i, int j) { return base + 1 + (i - 1) * n_lon + (j % n_lon); };
  for (int j = 0; j < n_lon; ++j) {
    t.insert(t.end(), {base, ring(1, j), ring(1, j + 1)});
    tm.push_back(mesh);
    t.insert(t.end(), {south, ring(n_lat - 1, j + 1), ring(n_lat - 1, j)});
    tm.push_back(mesh);
  }
  for (int i = 1; i + 1 < n_lat; ++i)
    for (int j = 0; j < n_lon; ++j) {
      t.insert(t.end(), {ring(i, j), ring(i + 1, j), ring(i + 1, j + 1)});
      tm.push_back(mesh);
      t.insert(t.end(), {ring(i, j), ring(i + 1, j + 1), ring(i, j + 1)});
      tm.push_back(mesh);
    }
}

// Every triangle sits in exactly one leaf, every reference is in range, the
// levels partition the nodes and the walk's stack bound holds.
static void check_hierarchy(const MeshHierarchy& H, long n_tri) {
  CHECK((long)H.tri.size() == n_tri && (long)H.tri_orig.size() == n_tri);
  std::vector<int> seen(n_tri, 0);
  for (long i = 0; i < n_tri; ++i) {
    CHECK(H.tri_orig[i] >= 0 && H.tri_orig[i] < n_tri);
    if (H.tri_orig[i] >= 0 && H.tri_orig[i] < n_tri) ++seen[H.tri_orig[i]];
  }
  for (long i = 0; i < n_tri; ++i) CHECK(seen[i] == 1);
  std::vector<int> covered(n_tri, 0);
  const int n = (int)H.nodes.size();
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < 4; ++j) {
      const int c = H.nodes[k].child[j];
      if (c == kEmptyChild) continue;
      if (c >= 0) {
        CHECK(c > k && c < n);   // breadth first: children after their parent
      } else {
        const int first = (~c) >> 4, cnt = (~c) & 15;
        CHECK(cnt >= 1 && cnt <= kLeafCap && first >= 0 && first + cnt <= n_tri);
        for (int i = first; i < first + cnt && i < n_tri; ++i) ++covered[i];
      }
    }
  for (long i = 0; i < n_tri; ++i) CHECK(covered[i] == 1);
  CHECK(!H.level_begin.empty() && H.level_begin.front() == 0 && H.level_begin.back() == n);
  for (size_t l = 1; l < H.level_begin.size(); ++l) CHECK(H.level_begin[l] > H.level_begin[l - 1]);
  CHECK(3 * H.depth <= kMaxBvhStack);
}

static void hierarchy_checks() {
  std::vector<double> v;
  std::vector<int32_t> t, tm;
  uv_sphere(0, 0, 0.03, 0.012, 40, 80, 0, v, t, tm);
  uv_sphere(0.002, 0, 0.031, 0.004, 12, 24, 1, v, t, tm);
  MeshHierarchy H;
  const long n_tri = (long)tm.size();
  CHECK(build_mesh_bvh(v.data(), (long)v.size() / 3, t.data(), tm.data(), n_tri, H) == 0);
  check_hierarchy(H, n_tri);
  // degenerate input: 300 copies of one triangle (coincident centroids, no
  // separating plane) must still give a valid hierarchy
  std::vector<double> v2 = {0, 0, 0.02, 0.001, 0, 0.02, 0, 0.001, 0.02};
  std::vector<int32_t> t2, tm2;
  for (int i = 0; i < 300; ++i) { t2.insert(t2.end(), {0, 1, 2}); tm2.push_back(0); }
  MeshHierarchy H2;
  CHECK(build_mesh_bvh(v2.data(), 3, t2.data(), tm2.data(), 300, H2) == 0);
  check_hierarchy(H2, 300);
  // a single triangle
  MeshHierarchy H3;
  CHECK(build_mesh_bvh(v2.data(), 3, t2.data(), tm2.data(), 1, H3) == 0);
  check_hierarchy(H3, 1);
}

// The windows of sum_pieces added in two different orders give the same
// words, and the read-out agrees with a long double sum.
static void sum_checks() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  std::uniform_int_distribution<int> ex(-60, 40);
  const int n = 20000;
  std::vector<double> x(n);
  long double ref = 0.0L;
  for (int i = 0; i < n; ++i) {
    x[i] = std::ldexp(u(rng), ex(rng));
    ref += (long double)x[i];
  }
  unsigned long long a[kSumWords] = {0}, b[kSumWords] = {0};
  auto add = [](unsigned long long* w, double v) {
    SumPieces p;
    if (!sum_pieces(v, &p)) return;
    if (p.over) { w[kSumBins] += 1; return; }
    w[p.b] += p.hi;
    w[p.b - 1] += p.lo;
  };
  for (int i = 0; i < n; ++i) add(a, x[i]);
  for (int i = n - 1; i >= 0; --i) add(b, x[i]);
  for (int k = 0; k < kSumWords; ++k) CHECK(a[k] == b[k]);
  const double got = sum_value(a);
  CHECK(std::fabs(got - (double)ref) <= 1e-9 * std::fabs((double)ref) + 1e-300);
  unsigned long long c[kSumWords] = {0};
  add(c, 1e300);   // beyond the last window: the total reads NaN
  CHECK(std::isnan(sum_value(c)));
  unsigned long long d[kSumWords] = {0};
  add(d, 1e-200);  // below the first window: dropped
  CHECK(sum_value(d) == 0.0);
}

// Argument checks of the C-ABI: every entry point rejects NULL handles and
// buffers with US_EINVAL and a message, before touching the device.
static void abi_checks() {
  us_ctx* ctx = nullptr;
  // no GPU in this process: creating a context fails cleanly
  const int rc = us_create(0, &ctx);
  CHECK(rc == US_OK || rc == US_EDEVICE);
  if (rc == US_OK) us_destroy(ctx);
  CHECK(us_create(0, nullptr) == US_EINVAL);
  us_probe_desc pd{};
  us_probe* probe = nullptr;
  CHECK(us_probe_upload(nullptr, &pd, &probe) == US_EINVAL && probe == nullptr);
  CHECK(us_last_error() != nullptr && us_last_error()[0] != 0);
  us_scene_desc sd{};
  us_scene* scene = nullptr;
  int32_t np = 0;
  CHECK(us_scene_upload(nullptr, &sd, &scene, &np) == US_EINVAL && scene == nullptr);
  CHECK(us_scene_set_params(nullptr, nullptr, 0, nullptr) == US_EINVAL);
  us_tx_desc tx{0.0, 0};
  float buf[16] = {0};
  CHECK(us_simulate_rf(nullptr, nullptr, nullptr, &tx, 1, 0, 1, 0, 1, 1, buf, nullptr, nullptr, buf,
                       sizeof(buf), nullptr) == US_EINVAL);
  CHECK(us_simulate_rf_workspace_size(nullptr, nullptr, 1, 1, 1) == 0);
  CHECK(us_beamform(nullptr, nullptr, nullptr, &tx, 1, buf, buf, buf, sizeof(buf), nullptr) == US_EINVAL);
  CHECK(us_bmode(nullptr, buf, 4, 60.0f, buf, buf, sizeof(buf), nullptr) == US_EINVAL);
  CHECK(us_bmode_vjp(nullptr, buf, buf, 4, 60.0f, buf, buf, sizeof(buf), nullptr) == US_EINVAL);
  double loss = 0.0;
  CHECK(us_image_loss(nullptr, buf, buf, 4, 0.0, 1.0, &loss, nullptr, buf, sizeof(buf), nullptr) == US_EINVAL);
  CHECK(us_beamform_vjp(nullptr, nullptr, nullptr, &tx, 1, buf, buf, buf, sizeof(buf), nullptr) == US_EINVAL);
  double g[4] = {0};
  CHECK(us_simulate_rf_vjp(nullptr, nullptr, nullptr, &tx, 1, 0, 1, 0, 1, 1, buf, g, buf, sizeof(buf),
                           nullptr) == US_EINVAL);
  CHECK(us_param_map(nullptr, g, g, g, 4, g, nullptr) == US_EINVAL);
  CHECK(us_adam_step(nullptr, g, g, g, g, g, g, g, 4, 1, 0.9, 0.999, 1e-8, 0.0, nullptr) == US_EINVAL);
  CHECK(us_destroy(nullptr) == US_EINVAL || us_destroy(nullptr) == US_OK);
  CHECK(us_probe_destroy(nullptr) == US_OK || us_probe_destroy(nullptr) == US_EINVAL);
  CHECK(us_scene_destroy(nullptr) == US_OK || us_scene_destroy(nullptr) == US_EINVAL);
}

int main() {
  hierarchy_checks();
  sum_checks();
  abi_checks();
  if (g_fail) {
    std::printf("%d host check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
