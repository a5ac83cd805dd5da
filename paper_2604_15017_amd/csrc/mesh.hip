// Closed triangle meshes (the anatomy scenes of Sec. 4): bounding-volume
// hierarchy built once on the host from the rest shape (binary tree by the
// binned surface-area heuristic, collapsed to 4-wide nodes by pulling up the
// grandchildren of the largest inner children), then refitted on the device
// whenever the displacement coefficients change, so that the topology stays
// fixed and only the boxes move. Nodes are numbered breadth first: the nodes
// of one depth form a contiguous range and a refit is one launch per depth,
// deepest first.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"

namespace usrt {

namespace {

struct Box {
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void add(const double* p) {
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p[k]); hi[k] = std::max(hi[k], p[k]); }
  }
  void add(const Box& b) {
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], b.lo[k]); hi[k] = std::max(hi[k], b.hi[k]); }
  }
  double area() const {
    const double x = hi[0] - lo[0], y = hi[1] - lo[1], z = hi[2] - lo[2];
    return (x < 0 || y < 0 || z < 0) ? 0.0 : 2.0 * (x * y + y * z + z * x);
  }
};

struct TmpNode {
  int left = -1, right = -1;   // children (temporary numbering), -1 for a leaf
  int first = 0, count = 0;    // leaf range in the permutation
  int depth = 0;
  double area = 0.0;           // surface area of the node's box
};

// 4-wide node before numbering: binary-tree ids of its children.
struct Wide {
  int slot[4];
  int n = 0;
  int depth = 0;
};

constexpr int kLeafMax = 2;
constexpr int kBins = 16;

struct Builder {
  const double* v;
  const int32_t* tris;
  std::vector<Box> tbox;
  std::vector<double> cen;      // [T][3]
  std::vector<int> perm;
  std::vector<TmpNode> nodes;
  int max_depth_seen = 0;

  // Split [first, first + count) at the best binned SAH plane; returns the
  // size of the left part (0 = make a leaf). *halve is set when no plane
  // separates the triangles and the range must be halved by the caller.
  bool too_deep = false;   // a leaf at the depth limit would exceed kLeafCap

  int split(int first, int count, const Box& bounds, int depth, bool* halve) {
    *halve = false;
    if (count <= kLeafMax) return 0;
    if (depth >= kMaxBvhDepth) {
      too_deep |= count > kLeafCap;
      return 0;
    }
    Box cb;
    for (int i = first; i < first + count; ++i) cb.add(&cen[3 * (size_t)perm[i]]);
    int axis = 0;
    double ext = cb.hi[0] - cb.lo[0];
    for (int k = 1; k < 3; ++k)
      if (cb.hi[k] - cb.lo[k] > ext) { ext = cb.hi[k] - cb.lo[k]; axis = k; }
    int* p = perm.data() + first;
    if (!(ext > 0.0)) {   // coincident centroids: halve by index
      *halve = true;
      return count / 2;
    }
    const double scale = kBins / ext;
    auto bin_of = [&](int t) {
      const int b = (int)((cen[3 * (size_t)t + axis] - cb.lo[axis]) * scale);
      return std::min(std::max(b, 0), kBins - 1);
    };
    int cnt[kBins] = {0};
    Box bb[kBins];
    for (int i = 0; i < count; ++i) {
      const int b = bin_of(p[i]);
      ++cnt[b];
      bb[b].add(tbox[p[i]]);
    }
    double right_area[kBins];
    int right_cnt[kBins];
    Box acc;
    int n = 0;
    for (int b = kBins - 1; b > 0; --b) {
      acc.add(bb[b]); n += cnt[b];
      right_area[b] = acc.area(); right_cnt[b] = n;
    }
    Box lacc;
    int ln = 0, best_b = -1;
    double best = INFINITY;
    for (int b = 1; b < kBins; ++b) {
      lacc.add(bb[b - 1]); ln += cnt[b - 1];
      if (ln == 0 || right_cnt[b] == 0) continue;
      const double c = lacc.area() * ln + right_area[b] * right_cnt[b];
      if (c < best) { best = c; best_b = b; }
    }
    if (best_b < 0) { *halve = true; return count / 2; }
    // cost model: one box test costs about one triangle test
    const double leaf_cost = bounds.area() * count;
    if (count <= kLeafCap && best + bounds.area() >= leaf_cost) return 0;
    int* mid = std::partition(p, p + count, [&](int t) { return bin_of(t) < best_b; });
    const int nl = (int)(mid - p);
    if (nl == 0 || nl == count) { *halve = true; return count / 2; }
    return nl;
  }

  int build(int first, int count, int depth) {
    const int id = (int)nodes.size();
    nodes.push_back(TmpNode{});
    nodes[id].depth = depth;
    max_depth_seen = std::max(max_depth_seen, depth);
    Box bounds;
    for (int i = first; i < first + count; ++i) bounds.add(tbox[perm[i]]);
    nodes[id].area = bounds.area();
    bool halve = false;
    const int nl = split(first, count, bounds, depth, &halve);
    if (halve) {
      // halving: order by centroid along the widest axis first so the halves are compact
      Box cb;
      for (int i = first; i < first + count; ++i) cb.add(&cen[3 * (size_t)perm[i]]);
      int axis = 0;
      for (int k = 1; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > cb.hi[axis] - cb.lo[axis]) axis = k;
      int* p = perm.data() + first;
      std::nth_element(p, p + nl, p + count, [&](int a, int b) {
        return cen[3 * (size_t)a + axis] < cen[3 * (size_t)b + axis];
      });
    }
    if (nl == 0) {
      nodes[id].first = first;
      nodes[id].count = count;
      return id;
    }
    const int l = build(first, nl, depth + 1);
    const int r = build(first + nl, count - nl, depth + 1);
    nodes[id].left = l;
    nodes[id].right = r;
    return id;
  }
};

}  // namespace

int build_mesh_bvh(const double* vertices, long n_vertices, const int32_t* tris,
                   const int32_t* tmesh, long n_tri, MeshHierarchy& out) {
  (void)n_vertices;
  Builder b{vertices, tris};
  b.tbox.resize(n_tri);
  b.cen.resize(3 * (size_t)n_tri);
  b.perm.resize(n_tri);
  for (long t = 0; t < n_tri; ++t) {
    Box& bx = b.tbox[t];
    for (int j = 0; j < 3; ++j) bx.add(vertices + 3 * (size_t)tris[3 * t + j]);
    for (int k = 0; k < 3; ++k) b.cen[3 * t + k] = 0.5 * (bx.lo[k] + bx.hi[k]);
    b.perm[t] = (int)t;
  }
  b.nodes.reserve(2 * (size_t)n_tri / kLeafMax + 16);
  b.build(0, (int)n_tri, 0);
  if (b.max_depth_seen > kMaxBvhDepth || b.too_deep) return -1;

  // collapse to 4-wide nodes: a node takes its two children, then repeatedly
  // replaces its inner child of largest area by that child's two children
  std::vector<TmpNode>& T = b.nodes;
  std::vector<Wide> W;
  auto leaf_ref = [&](int id) { return ~((T[id].first << 4) | T[id].count); };
  auto make_wide = [&](int bin, int depth) {
    Wide w;
    w.depth = depth;
    if (T[bin].left < 0) {          // a single leaf as the whole tree
      w.slot[0] = bin;
      w.n = 1;
    } else {
      w.slot[0] = T[bin].left;
      w.slot[1] = T[bin].right;
      w.n = 2;
      while (w.n < 4) {
        int best = -1;
        for (int j = 0; j < w.n; ++j)
          if (T[w.slot[j]].left >= 0 && (best < 0 || T[w.slot[j]].area > T[w.slot[best]].area)) best = j;
        if (best < 0) break;
        const int x = w.slot[best];
        w.slot[best] = T[x].left;
        w.slot[w.n++] = T[x].right;
      }
    }
    W.push_back(w);
    return (int)W.size() - 1;
  };
  make_wide(0, 0);
  // breadth first: the children of node i are created while node i is read
  std::vector<int> wchild;   // per wide node, 4 entries: wide id of an inner slot, or -1
  for (size_t i = 0; i < W.size(); ++i) {
    for (int j = 0; j < 4; ++j) wchild.push_back(-1);
    for (int j = 0; j < W[i].n; ++j) {
      const int x = W[i].slot[j];
      if (T[x].left >= 0) {
        const int w = make_wide(x, W[i].depth + 1);
        wchild[4 * i + j] = w;
      }
    }
  }
  // breadth-first numbering (creation order is already breadth first)
  const int n = (int)W.size();
  out.level_begin.assign(1, 0);
  for (int i = 1; i < n; ++i)
    if (W[i].depth != W[i - 1].depth) out.level_begin.push_back(i);
  out.level_begin.push_back(n);
  out.nodes.resize(n);
  for (int k = 0; k < n; ++k) {
    BvhNode& nd = out.nodes[k];
    for (int j = 0; j < 4; ++j) {
      nd.lox[j] = nd.loy[j] = nd.loz[j] = nd.hix[j] = nd.hiy[j] = nd.hiz[j] = kFarBox;
      nd.pad[j] = 0;
      if (j >= W[k].n) nd.child[j] = kEmptyChild;
      else if (wchild[4 * k + j] >= 0) nd.child[j] = wchild[4 * k + j];
      else nd.child[j] = leaf_ref(W[k].slot[j]);
    }
  }
  out.depth = (int)out.level_begin.size() - 1;
  if (3 * out.depth > kMaxBvhStack) return -1;
  out.tri.resize(n_tri);
  out.tri_orig.resize(n_tri);
  for (long i = 0; i < n_tri; ++i) {
    const int t = b.perm[i];
    out.tri[i] = make_int4(tris[3 * (size_t)t], tris[3 * (size_t)t + 1], tris[3 * (size_t)t + 2], tmesh[t]);
    out.tri_orig[i] = t;
  }
  return 0;
}

namespace {

// v = v_rest + (sum_j q[mesh(v)][j] phi_j(v)) n(v)
__global__ __launch_bounds__(256) void k_mesh_vertices(long n_v, const double* __restrict__ vrest,
                                                       const double* __restrict__ vnormal,
                                                       const double* __restrict__ vbasis,
                                                       const int* __restrict__ vmesh, int n_basis,
                                                       const double* __restrict__ q,
                                                       double* __restrict__ vcur) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_v) return;
  const double* qm = q + (long)vmesh[v] * n_basis;
  const double* phi = vbasis + v * n_basis;
  double s = 0.0;
  for (int j = 0; j < n_basis; ++j) s += qm[j] * phi[j];
  for (int k = 0; k < 3; ++k) vcur[3 * v + k] = vrest[3 * v + k] + s * vnormal[3 * v + k];
}

__device__ __forceinline__ float round_down(double x) {
  const float f = (float)x;
  return (double)f > x ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float round_up(double x) {
  const float f = (float)x;
  return (double)f < x ? nextafterf(f, INFINITY) : f;
}

// Child boxes of the inner nodes [begin, end) of one depth: a leaf child's
// from its triangles' current vertices (fp64, padded by kBoxPad and rounded
// outward to fp32), an
// inner child's as the union of its own two boxes, which belong to a deeper
// level and are already refitted.
__device__ __forceinline__ void child_box(const BvhNode* nodes, int ref, const int4* tri,
                                          const double* vcur, float* lo, float* hi) {
  if (ref == kEmptyChild) {   // unused slot: a point far away
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = kFarBox;
    return;
  }
  if (ref >= 0) {   // union of the used slots of an inner child (refitted one level deeper)
    const BvhNode c = nodes[ref];
    for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int j = 0; j < 4; ++j) {
      if (c.child[j] == kEmptyChild) continue;
      lo[0] = fminf(lo[0], c.lox[j]); lo[1] = fminf(lo[1], c.loy[j]); lo[2] = fminf(lo[2], c.loz[j]);
      hi[0] = fmaxf(hi[0], c.hix[j]); hi[1] = fmaxf(hi[1], c.hiy[j]); hi[2] = fmaxf(hi[2], c.hiz[j]);
    }
    return;
  }
  double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
  const int first = (~ref) >> 4, cnt = (~ref) & 15;
  for (int t = first; t < first + cnt; ++t) {
    const int4 tv = tri[t];
    const int id[3] = {tv.x, tv.y, tv.z};
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        const double c = vcur[3 * (long)id[j] + k];
        l[k] = fmin(l[k], c);
        h[k] = fmax(h[k], c);
      }
  }
  for (int k = 0; k < 3; ++k) {
    lo[k] = round_down(l[k] - (double)kBoxPad);
    hi[k] = round_up(h[k] + (double)kBoxPad);
  }
}

__global__ __launch_bounds__(256) void k_refit(BvhNode* __restrict__ nodes, int begin, int end,
                                               const int4* __restrict__ tri,
                                               const double* __restrict__ vcur) {
  const int i = begin + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= end) return;
  BvhNode nd = nodes[i];
  for (int j = 0; j < 4; ++j) {
    float lo[3], hi[3];
    child_box(nodes, nd.child[j], tri, vcur, lo, hi);
    nd.lox[j] = lo[0]; nd.loy[j] = lo[1]; nd.loz[j] = lo[2];
    nd.hix[j] = hi[0]; nd.hiy[j] = hi[1]; nd.hiz[j] = hi[2];
  }
  nodes[i] = nd;
}

// Leaf-order triangle records from the current vertices.
__global__ __launch_bounds__(256) void k_trec(long n_tri, const int4* __restrict__ tri,
                                              const double* __restrict__ vcur, TriRec* __restrict__ rec) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_tri) return;
  const int4 tv = tri[i];
  TriRec r;
  for (int k = 0; k < 3; ++k) {
    const double p0 = vcur[3 * (long)tv.x + k];
    r.p0[k] = p0;
    r.e1[k] = vcur[3 * (long)tv.y + k] - p0;
    r.e2[k] = vcur[3 * (long)tv.z + k] - p0;
  }
  r.pad = 0.0;
  rec[i] = r;
}

}  // namespace

void launch_mesh_refit(const MeshDevice& m, const double* q, hipStream_t s) {
  if (m.n_vertices > 0)
    hipLaunchKernelGGL(k_mesh_vertices, dim3((unsigned)((m.n_vertices + 255) / 256)), dim3(256), 0, s,
                       m.n_vertices, m.vrest, m.vnormal, m.vbasis, m.vmesh, m.n_basis, q, m.vcur);
  if (m.n_triangles > 0)
    hipLaunchKernelGGL(k_trec, dim3((unsigned)((m.n_triangles + 255) / 256)), dim3(256), 0, s,
                       m.n_triangles, m.tri, m.vcur, m.trec);
  for (int lv = (int)m.level_begin.size() - 2; lv >= 0; --lv) {
    const int b = m.level_begin[lv], e = m.level_begin[lv + 1];
    hipLaunchKernelGGL(k_refit, dim3((unsigned)((e - b + 255) / 256)), dim3(256), 0, s, m.nodes, b, e,
                       m.tri, m.vcur);
  }
}

}  // namespace usrt
