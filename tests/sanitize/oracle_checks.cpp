// The FP64 oracle's transport built with AddressSanitizer and
// UndefinedBehaviorSanitizer: one small scene with every surface kind (two
// planes, a diffuse sphere, a rough cylinder, a closed triangle mesh) traced
// forward, with its dual-number gradient, decision hashes and recorded branch
// probabilities. Exits non-zero on a failed check; the sanitizers abort on
// the first report.
#include "../../oracle/transport.cpp"

#include <cstdio>
#include <vector>

int main() {
  int fails = 0;
  // regions: 0 water, 1 tissue, 2 sphere, 3 cylinder, 4 mesh inside
  const int n_regions = 5;
  std::vector<int32_t> plane_regions = {0, 1, 1, 0};
  std::vector<double> plane_kd = {0.0, 0.1};
  std::vector<int32_t> sphere_regions = {2, 1};
  std::vector<double> sphere_kd = {0.5};
  std::vector<int32_t> cyl_regions = {3, 1};
  std::vector<double> cyl_kd = {0.2};
  // an octahedron around (0, 0, 22 mm) as the closed mesh, one basis function
  const double c = 0.022, r = 0.002;
  std::vector<double> vrest = {r, 0, c, -r, 0, c, 0, r, c, 0, -r, c, 0, 0, c + r, 0, 0, c - r};
  std::vector<double> vnormal = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
  std::vector<double> vbasis(6, 1.0);
  std::vector<int32_t> vmesh(6, 0);
  std::vector<int32_t> tris = {0, 2, 4, 2, 1, 4, 1, 3, 4, 3, 0, 4, 2, 0, 5, 1, 2, 5, 3, 1, 5, 0, 3, 5};
  std::vector<int32_t> tmesh(8, 0);
  std::vector<int32_t> mesh_regions = {4, 1};
  std::vector<double> mesh_kd = {0.3};
  OrSceneDesc sd{};
  sd.n_regions = n_regions;
  sd.n_planes = 2;
  sd.n_spheres = 1;
  sd.plane_regions = plane_regions.data();
  sd.plane_kd = plane_kd.data();
  sd.sphere_regions = sphere_regions.data();
  sd.sphere_kd = sphere_kd.data();
  sd.start_region = 0;
  sd.n_meshes = 1;
  sd.n_basis = 1;
  sd.mesh_regions = mesh_regions.data();
  sd.mesh_kd = mesh_kd.data();
  sd.n_vertices = 6;
  sd.n_triangles = 8;
  sd.vrest = vrest.data();
  sd.vnormal = vnormal.data();
  sd.vbasis = vbasis.data();
  sd.vmesh = vmesh.data();
  sd.tris = tris.data();
  sd.tmesh = tmesh.data();
  sd.n_cylinders = 1;
  sd.cylinder_regions = cyl_regions.data();
  sd.cylinder_kd = cyl_kd.data();
  // theta: regions (c, Z, alpha), plane depths, sphere (x, y, z, r), cylinder
  // (x, z, R), roughness of planes, sphere, cylinder, mesh, mesh coefficient
  std::vector<double> theta = {1480, 1.48, 0.0, 1540, 1.63, 0.5, 1580, 1.7, 0.7, 1560, 1.8, 0.6,
                               1600, 1.75, 0.8, 0.008, 0.040, 0.004, 0.0, 0.015, 0.0015, -0.004, 0.030,
                               0.002, 0.05, 0.0, 0.1, 0.2, 0.15, 0.0};
  OrProbeDesc pd{32, 3e-4, 3e-4, 5e-3, 5e6, 2.0, 40e6, 2048, 1540.0, 20 * M_PI / 180, 60 * M_PI / 180};
  const double angles[2] = {-0.1, 0.12};
  const uint32_t ids[2] = {0, 1};
  std::vector<double> probs(2 * 32 * 64 * 6, 0.0);
  OrRunDesc rd{2, angles, ids, 5, 64, 0, 32 * 64, 6, 0, 2, 1, probs.data()};
  std::vector<uint64_t> hashes(2 * 32 * 64, 0);
  std::vector<double> g_h(2 * 32 * 2048);
  for (size_t i = 0; i < g_h.size(); ++i) g_h[i] = std::sin(0.001 * (double)i);
  std::vector<int32_t> sel;
  for (int j = 0; j < (int)theta.size(); ++j) sel.push_back(j);
  void* h = oracle_trace(&sd, &pd, &rd, theta.data(), g_h.data(), sel.data(), (int)sel.size(), hashes.data());
  if (!h) { std::printf("FAILED: trace rejected its arguments\n"); return 1; }
  const int64_t n = oracle_result_count(h);
  if (n <= 0) { std::printf("FAILED: no contributions\n"); ++fails; }
  std::vector<int32_t> tx(n), el(n);
  std::vector<double> t(n), a(n), g(sel.size());
  std::vector<int64_t> ray(n);
  oracle_result_copy(h, tx.data(), el.data(), t.data(), a.data(), ray.data(), g.data());
  for (double x : g)
    if (!std::isfinite(x)) { std::printf("FAILED: non-finite gradient\n"); ++fails; break; }
  std::vector<double> hist(2 * 32 * 2048, 0.0);
  oracle_splat(n, tx.data(), el.data(), t.data(), a.data(), 32, 2048, pd.fs, hist.data());
  oracle_result_free(h);
  // the same rays again with the recorded probabilities, no gradient
  rd.prob_mode = 2;
  void* h2 = oracle_trace(&sd, &pd, &rd, theta.data(), nullptr, nullptr, 0, nullptr);
  if (!h2 || oracle_result_count(h2) != n) { std::printf("FAILED: replay with recorded probabilities\n"); ++fails; }
  if (h2) oracle_result_free(h2);
  // bad arguments are refused
  if (oracle_trace(nullptr, &pd, &rd, theta.data(), nullptr, nullptr, 0, nullptr) != nullptr) ++fails;
  std::printf(fails ? "oracle checks failed\n" : "oracle checks passed (%ld contributions)\n", (long)n);
  return fails ? 1 : 0;
}
