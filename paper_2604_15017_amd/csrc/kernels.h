// Internal interface between the C-ABI (api.hip) and the kernels.
#pragma once

#include <vector>

#include "common.h"

namespace usrt {

// Live-ray queue, structure of arrays (coalesced per field).
struct RayQueue {
  double *ox, *oy, *oz, *dx, *dy, *dz, *t, *w;
  uint32_t* rid;
  uint32_t* meta;   // region (8 bits) | last event not diffuse << 8 | transmit (local) << 12
};
constexpr size_t kRayQueueBytesPerRay = 8 * sizeof(double) + 2 * sizeof(uint32_t);

// Secondary-ray queue.
// Receiver-directed secondary ray queued by the bounce kernel: one 64-byte
// record (written and read as four 16-byte pieces, moved whole by the sort).
struct alignas(16) SecRec {
  double x, y, z, t, amp;
  uint32_t rid;
  uint32_t meta;   // region (8 bits) | element << 8
  uint32_t txk;    // transmit (local, 16 bits) | interaction index << 16
  uint32_t key;    // sort key (scenes that sort their receiver segments), else 0
  uint32_t rank;   // the record's place among those of its key (likewise)
  uint32_t pad;
};
static_assert(sizeof(SecRec) == 64, "secondary record layout");
struct SecondaryQueue {
  SecRec* rec;
};
constexpr size_t kSecondaryBytesPerRay = sizeof(SecRec);

// Receiver segments are marched in the order of a key, so that a wave takes
// segments that run close together through the same part of the hierarchy
// (in queue order its 64 segments head for random elements from scattered
// origins, and the wave waits for its longest walk): the cell of the origin
// on a kSortCellsZ x kSortCellsX grid over x in [x0, x0 + kSortCellsX /
// inv_dx) and z in [0, kSortCellsZ / inv_dz) (points outside go to the edge
// cells), then the target element. keys = 0: queue order.
constexpr int kSortCellsX = 64, kSortCellsZ = 64;
constexpr int kSortBlocks = 256;   // tiles of the offsets' scan
struct SegSort {
  int keys;               // cells x n_elem
  int n_elem;
  double x0, inv_dx, inv_dz;
  __device__ __forceinline__ uint32_t key(double x, double z, int e2) const {
    const int cx = (int)fmin(fmax(floor((x - x0) * inv_dx), 0.0), (double)(kSortCellsX - 1));
    const int cz = (int)fmin(fmax(floor(z * inv_dz), 0.0), (double)(kSortCellsZ - 1));
    return ((uint32_t)cz * kSortCellsX + (uint32_t)cx) * (uint32_t)n_elem + (uint32_t)e2;
  }
};
// count[0..n) -> its exclusive prefix sums, in place (part: kSortBlocks words).
void launch_sort_offsets(uint32_t* count, int n, uint32_t* part, hipStream_t s);

struct TraceArgs {
  SceneView scene;
  ProbeView probe;
  TxTable tx;             // the transmits of this launch group
  uint64_t seed;
  int rays_per_elem;
  int max_bounces;
  long ray_begin, ray_count;
  long g0, n_chunk;       // chunk of the flattened (local transmit, ray) index space
  int tx_base;            // index of the group's first transmit in the caller's list
  RayQueue qin, qout;
  SecondaryQueue nee;
  // counts[k], k = 1..max_bounces + 1: rays alive after interaction k (low 32
  // bits) and secondary rays spawned at interaction k (high 32 bits)
  unsigned long long* counts;
  long long* h;           // deposit histogram [n_tx][n_elem][n_t], units of 1 / hist_scale
  double hist_scale;
  unsigned long long* hist_over;   // count of clamped deposit weights
  // deposits of the secondary rays recorded for the binned splat in
  // kDepShards shards of dep_cap / kDepShards records (shard = block index
  // mod kDepShards, count dep_count[shard]); beyond a shard's capacity (or
  // with dep_cap = 0) they are added to h directly
  DepositList dep;
  long dep_cap;
  unsigned long long* dep_count;
  unsigned long long* counters;   // optional int64[5]
  unsigned long long* hash;       // optional [n_tx][ray_count]
  // With sort.keys > 0 the receiver segments of each interaction are
  // marched in key order: the bounce kernel counts the keys in
  // sort_count[sort.keys] (zeroed before it) and keeps each record's rank
  // among its key's; launch_secondary_sort turns the counts into offsets
  // (sort_part: kSortBlocks words) and writes the permutation sort_perm
  // (record index in key order, over the interaction's dead input queue).
  SegSort sort;
  uint32_t* sort_count;
  uint32_t* sort_part;
  uint32_t* sort_perm;
};

// Step record of the replay: the exact state before step k of a ray and the
// surface the step hits (80 bytes, written and read as five 16-byte pieces,
// so that records scattered by chunk ray still move whole sectors).
struct alignas(16) StepRec {
  double ox, oy, oz, dx, dy, dz, t, w;
  double L;          // distance to the surface hit
  uint32_t meta;     // region | last event not diffuse << 8 | hit kind << 12
  int hidx;          // hit index (leaf-order triangle for meshes)
};
// Adjoints of the inputs of the secondary ray of a diffuse interaction:
// x, n_r, A_r, w_att, t' (80 bytes with the padding).
struct alignas(16) StepAdj {
  double xb, yb, zb, nxb, nyb, nzb, Ab, wb, tb, pad;
};
static_assert(sizeof(StepRec) == 80 && sizeof(StepAdj) == 80, "replay record layout");

// Records of one chunk of rays: step k of chunk ray i at [(k - 1) * cap + i].
struct ReplayStack {
  StepRec* rec;
  StepAdj* adj;
  int* last;                                     // [cap] last step that can carry a deposit
  uint32_t* queue;          // [max_bounces][cap]: chunk rays of the diffuse interactions of step k
  unsigned long long* queue_begin;   // [max_bounces + 1]: exclusive prefix of the step sizes
  // with ReplayArgs::sort.keys > 0: each queued interaction's (key, rank
  // among the step's entries of that key) [max_bounces][cap], and the queue
  // in key order within each step, indexed like queue_begin
  uint2* sort_kr;
  uint32_t* sort_q;
};
constexpr int kMaxReplayBlocks = 2048;
// The receiver segments of the queued diffuse interactions as a recorded
// forward marched them, arrays over the queue index q < cap: the state with
// the crossing count (n_cross << 2 | state; state 0: no segment, facing away
// or outside the directivity; 1: blocked; 2: reached the element), the
// march's sums, and its first kMarchLegs crossings (distance from the
// origin, hit word), crossing j of entry q at [j * cap + q]. Crossings past
// a segment's count are not written, and lanes of a wave (consecutive q)
// touch consecutive words.
constexpr int kMarchLegs = 8;
struct MarchRecs {
  double* tof;
  double* att;
  double* trans;
  uint32_t* nstate;
  double* s;
  int* h;
  long cap;   // 0: no records
};
constexpr long kMarchPerRay = 4;   // march records per ray of a recorded frame (more are marched again)

struct ReplayArgs {
  SceneView scene;
  ProbeView probe;
  TxTable tx;
  uint64_t seed;
  int rays_per_elem;
  int max_bounces;
  long ray_begin, ray_count;
  long g0;                // first ray of the chunk within the transmit group
  long cap;               // chunk capacity (rays)
  int tx_base;
  int n_params;
  int n_grad;             // leading theta entries summed in LDS (regions, planes, spheres, cylinders, roughness)
  int grad_copies;        // interleaved LDS copies of those sums (power of two, <= 16; set by the launchers)
  const float* gh;        // dL/dh [n_tx][n_elem][n_t]
  unsigned long long* g_sum;   // [n_grad][kSumWords] accumulators of the gradient (zeroed per call)
  unsigned long long* vadj;    // [kVadjCopies][kSumWords][vadj_stride] mesh vertex adjoints along vnormal (zeroed per call)
  long vadj_stride;
  ReplayStack stk;
  // receiver segments of the secondary phase in key order (as the forward
  // marches them): counts per (step, key) [max_bounces][sort.keys], zeroed
  // before the forward phase, then offsets (sort_part: kSortBlocks words)
  SegSort sort;
  uint32_t* sort_count;
  uint32_t* sort_part;
  RayQueue qin, qout;     // live rays of the forward phase (rid holds the chunk index)
  unsigned long long* counts;   // [max_bounces + 2]: survivors of step k | diffuse interactions << 32
  // optional (null): d/d steering angle of each transmit (tx_base + local
  // index), then d/d c_ref, d/d pitch and d/d f0, accumulated by
  // launch_grad_finish from acq_sum ([n_tx_total + 3][kSumWords], zeroed per
  // call); n_tx_total entries of angles precede the three. With g_acq, gh_f0
  // holds the rows of dL/dh for the pulse's derivative in f0 (the f0 entry
  // gets each deposit's amplitude times gh_f0 at its time; the attenuation's
  // share of d/d f0 is added by launch_grad_finish)
  double* g_acq;
  unsigned long long* acq_sum;
  const float* gh_f0;
  int n_tx_total;
  // a recorded forward (null otherwise): the forward phase adds the array
  // hits' deposits and launch_replay_deposit the receiver segments' to h, in
  // units of 1 / hist_scale, as the forward transport does
  long long* h;
  double hist_scale;
  unsigned long long* hist_over;
  // a recorded frame (cap 0 otherwise): the march of queued interaction q
  // (q < march.cap), written by launch_replay_deposit and read by the
  // secondary phase in place of marching again
  MarchRecs march;
  // a recorded forward, optional (null): the event counters of the forward
  // transport (int64[5], accumulated), counted by the forward phase's
  // deposit variant and by launch_replay_deposit
  unsigned long long* counters;
};
// The three phases of the replay over chunk rays [0, n): the forward phase
// once per step k = 1..max_bounces + 1 (queues swapped in between), the
// prefix over the per-step interaction counts, the secondary phase, then the
// reverse sweep. The counts must be zero before the forward step k = 1. The
// analytic gradient collects in g_sum; add it to g_theta with
// launch_grad_finish once all chunks are done.
void launch_replay_forward(const ReplayArgs& a, int k, long n, hipStream_t s);
// The receiver segments of the queued diffuse interactions deposited into a.h
// (a recorded forward; after launch_replay_prefix and launch_replay_sort).
void launch_replay_deposit(const ReplayArgs& a, long max_entries, hipStream_t s);
void launch_replay_prefix(const ReplayArgs& a, hipStream_t s);
void launch_replay_secondary(const ReplayArgs& a, long max_entries, hipStream_t s);
// With sort.keys > 0, after the prefix: the queue in key order (stk.sort_q).
void launch_replay_sort(const ReplayArgs& a, long max_entries, hipStream_t s);
void launch_replay_reverse(const ReplayArgs& a, long n, hipStream_t s);
// g_theta[j] += total of g_sum entry j (j < n_grad); with g_acq, also
// g_acq[i] += total of acq_sum entry i (i < n_acq), the f0 entry f0_at taking
// sum_r theta[3 r + 2] (total of entry 3 r + 2) inv_f0 besides.
void launch_grad_finish(const unsigned long long* g_sum, int n_grad, double* g_theta,
                        const unsigned long long* acq_sum, int n_acq, double* g_acq, int f0_at,
                        const double* theta, int n_regions, double inv_f0, hipStream_t s);
// Copies of the vertex adjoints: block b adds into copy b % kVadjCopies.
// Blocks are dealt round-robin to the eight XCDs, so each copy is updated
// from one XCD (its atomics meet in that XCD's L2), and four copies per XCD
// spread the blocks contending for a line. The copies are added up by
// launch_basis_gather. Within a copy the sums are word-major (word w of every
// vertex, then word w + 1): a value touches the two words of its magnitude's
// windows, and the vertex adjoints of one call span few windows, so the lines
// the atomics touch are those few rows of the copy rather than every vertex's
// whole accumulator.
constexpr int kVadjCopies = 32;
// vval[v] = total of vertex v over the copies, then
// g_q[m * n_basis + j] += sum_{v in mesh m} vval[v] vbasis[v][j].
void launch_basis_gather(const unsigned long long* vadj, long stride, long n_vertices, double* vval,
                         const double* vbasis, const long* vbeg, int n_meshes, int n_basis, double* g_q,
                         hipStream_t s);

// ---------------------------------------------------------------- inverse loop
void launch_param_map(const double* u, const double* lo, const double* hi, int n, double* theta,
                      hipStream_t s);
void launch_adam(double* u, double* m, double* v, const double* g, const double* lo, const double* hi,
                 const double* lr, int n, int step, double b1, double b2, double eps, double max_norm,
                 hipStream_t s);

// ---------------------------------------------------------------- meshes
// Hierarchy as built on the host (breadth-first nodes, leaf-order triangles).
struct MeshHierarchy {
  std::vector<BvhNode> nodes;
  std::vector<int4> tri;
  std::vector<int> tri_orig;
  std::vector<int> level_begin;   // inner nodes of depth l: [level_begin[l], level_begin[l + 1])
  int depth = 0;                  // number of inner levels of the 4-wide tree
};
// Returns 0, or -1 if the binary tree would exceed kMaxBvhDepth (or a leaf at
// that depth would hold more than kLeafCap triangles), or the 4-wide walk
// would need more than kMaxBvhStack stack entries.
int build_mesh_bvh(const double* vertices, long n_vertices, const int32_t* tris,
                   const int32_t* tmesh, long n_tri, MeshHierarchy& out);

// Device arrays of a scene's meshes.
struct MeshDevice {
  long n_vertices = 0, n_triangles = 0;
  int n_basis = 0;
  const double* vrest = nullptr;
  const double* vnormal = nullptr;
  const double* vbasis = nullptr;
  const int* vmesh = nullptr;
  double* vcur = nullptr;
  TriRec* trec = nullptr;
  BvhNode* nodes = nullptr;
  const int4* tri = nullptr;
  const long* vbeg = nullptr;     // [n_meshes + 1] vertex range of each mesh
  std::vector<int> level_begin;
};
// Current vertices from the displacement coefficients q (device,
// [n_meshes][n_basis]), then the boxes, deepest level first.
void launch_mesh_refit(const MeshDevice& m, const double* q, hipStream_t s);
void launch_fill_u32(uint32_t* p, long n, uint32_t v, hipStream_t s);

// Binned splat of the recorded deposits of rows [row0, row0 + n_rows)
// (n_rows <= kMaxBinRows, n_t < kMaxBinSamples): counting sort by row into
// `sorted`, then one block per row and time tile sums the row's deposits in
// LDS and adds the tile to h.
size_t splat_scratch_bytes(int n_rows);
void launch_splat_bin(const DepositList& dep, const unsigned long long* shard_count, long shard_cap,
                      int n_rows, uint4* sorted, void* scratch, hipStream_t s);
void launch_splat_accumulate(const uint4* sorted, const void* scratch, uint32_t row0, int n_rows,
                             int n_t, long long* h, double hist_scale, unsigned long long* hist_over,
                             hipStream_t s);
// The last chunk of a transmit group, fused with the pulse: each row of h
// (direct deposits and earlier chunks) plus the row's binned deposits, read
// out and filtered straight into rf. Returns -1 (nothing launched) when
// n_t > 8192 or the pulse is too long for the one-row-per-block layout.
int launch_splat_pulse(const uint4* sorted, const void* scratch, uint32_t row0, int n_rows, int n_t,
                       const long long* h, double hist_scale, unsigned long long* hist_over, const float* taps,
                       int M, float* rf, hipStream_t s);
void launch_bounce(const TraceArgs& a, int k, long max_rays, bool audit, hipStream_t s);
void launch_secondary(const TraceArgs& a, int k, long max_rays, bool audit, hipStream_t s);
// Counting sort of interaction k's receiver segments by key into sort_perm
// (with sort_keys > 0); launch_secondary then marches them in that order.
void launch_secondary_sort(const TraceArgs& a, int k, long max_rays, hipStream_t s);
int launch_pulse(const float* h, float* rf, const float* taps, int M, int n_t, long n_rows,
                 hipStream_t s);
// The same FIR from the fixed-point histogram: samples h / hist_scale (NaN
// everywhere when *hist_over is nonzero).
int launch_pulse_fixed(const long long* h, double hist_scale, const unsigned long long* hist_over, float* rf,
                       const float* taps, int M, int n_t, long n_rows, hipStream_t s);

// ---------------------------------------------------------------- image chain
struct GridView {
  int n_x, n_z;
  double x0, dx, z0, dz;
};

int launch_analytic(const float* rf, float2* A, const float2* twiddle, int n_t, long n_rows,
                    hipStream_t s);
void launch_das(const float2* A, float2* iq, const ProbeView& p, const GridView& g,
                const TxTable& tx, int n_tx_group, int tx_base, bool accumulate, hipStream_t s);
void launch_env_max(const float2* iq, long n_px, unsigned long long* key, hipStream_t s);
void launch_bmode(const float2* iq, long n_px, float dr_db, const unsigned long long* key,
                  float* bmode, hipStream_t s);
// sum: an order-independent accumulator of kSumWords words, zeroed by the caller
void launch_bmode_vjp(const float2* iq, const float* g_b, long n_px, float dr_db,
                      const unsigned long long* key, unsigned long long* sum, float2* g_iq, hipStream_t s);
void launch_bmode_vjp_fix(const float2* iq, long n_px, const unsigned long long* key,
                          const unsigned long long* sum, float2* g_iq, hipStream_t s);
// Gradients of the image with respect to the acquisition parameters (the
// steering angles, c_ref, the pitch): per-tile partial rows in part
// ([n_tx_group][das_acq_tiles][3] doubles), then added into out[n_tx_total + 2]
// (angles at tx_base.., c_ref, pitch), which the caller zeroes first.
long das_acq_tiles(const GridView& g);
void launch_das_acq(const float2* A, const float2* g_iq, const ProbeView& p, const GridView& g, const TxTable& tx,
                    int n_tx_group, int tx_base, int n_tx_total, double* part, double* out, hipStream_t s);
void launch_das_adjoint(const float2* g_iq, float2* g_A, const ProbeView& p, const GridView& g,
                        const TxTable& tx, int n_tx_group, int tx_base, hipStream_t s);
int launch_analytic_adjoint(const float2* g_A, float* g_rf, const float2* twiddle, int n_t,
                            long n_rows, hipStream_t s);
// launch_analytic_adjoint followed by launch_pulse_adjoint with the same
// reversed taps, in one kernel per RF row (the real row between them stays in
// LDS): g_h = P^T Re(T g_A), bit for bit the two-launch result.
int launch_analytic_pulse_adjoint(const float2* g_A, float* g_h, const float2* twiddle, const float* taps_reversed,
                                  int M, int n_t, long n_rows, hipStream_t s);
// acc: an order-independent accumulator of kSumWords words, zeroed by the caller
void launch_image_loss(const float* b, const float* ref, long n, double l1, double l2,
                       unsigned long long* acc, double* loss, float* gb, hipStream_t s);
int launch_pulse_adjoint(const float* g_rf, float* g_h, const float* taps, int M, int n_t,
                         long n_rows, hipStream_t s);

}  // namespace usrt
