// Batched blocked QB: many independent problems (Figure 4, P = 0) advanced
// together, one launch per step of the block loop for every active problem.
//
// Each block iteration runs, for all problems still active:
//   sketch -> Y = R Omega -> CholQR2 (Gram, Cholesky + inverse, apply) ->
//   [k > 0: C = Qbar^T Q, Q -= Qbar C, CholQR2] -> B_i = Q_i^T R with
//   ||B_i||^2 -> R -= Q_i B_i with ||R||^2 -> per-problem compensated sums
//   -> the stopping rule of qb_factor (Section 4.2) for each problem.
// The loop is planned on the device: a plan kernel turns each problem's
// state (rank k, width w, active) into the descriptors of every step, the
// products walk the units the plan counted (a fixed grid per launch), and a
// stop kernel applies the rule and sets the next width.  All launches of
// an iteration therefore have fixed arguments; eight iterations are
// captured once per call in a HIP graph, which is replayed until no
// problem is active (the host reads one flag per replay).  With the
// profiler on, or QB_BATCHED_EAGER set, the same launches run eagerly, one
// iteration at a time.  Problems stop independently; a product's units
// cover only the active problems.  Products use MFMA tiles of a class
// chosen per product role and panel width (a table, see g_tile), one launch
// per class the batch can use, with a unit -> (problem, tile, depth chunk)
// mapping; the Cholesky runs one workgroup per problem.  Inputs are float;
// every stored value and every product is float64, so each problem follows
// the float64 oracle.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/qb.h"
#include "qb_internal.hpp"

namespace qb {
namespace {

static_assert(kTile64 == QB_TILE_64X64 && kTileG16 == QB_TILE_16X16 &&
                  kTileG32 == QB_TILE_32X32 && kTileN32 == QB_TILE_64X32 &&
                  kTileM32 == QB_TILE_32X64 && kTileClasses == 5,
              "public tile class numbers");

constexpr double kDeltaRelB = 1e-13;   // hybrid band, relative to ||A||_F^2
constexpr double kFloorRelB = 0x1p-46;  // rounding floor of the residual, rel. ||A||_F
constexpr int kBMax = 64;               // widest panel of the batched form
constexpr int kKeptStride = kBMax + 2;  // ints per problem in the kept table
constexpr int kScal = 8;                // doubles per problem in the scalar table
// Depth split of the products whose output has few tiles (the w x w Gram,
// C = Qbar^T Q_i, B_i, and the m x w panels): a problem's product is cut
// into at most ceil(kSplitTiles / tiles) depth chunks of at least
// kSplitChunk, so that it spreads over about kSplitTiles workgroups; the
// chunks are then summed in order.  The depth loops bound the time of these
// products once few problems are left (measured on 512 uneven problems: a
// target of 16 -> 64 workgroups cut the batch from 285 to 257 ms and its
// longest problem alone from 69 to 45 ms; with the device-planned loop,
// 64 -> 128 cut the batch from 227.3 to 225.5 ms and the longest problem
// alone from 36.8 to 32.2 ms; 256 gave no further gain).  The choice
// depends only on the problem's own sizes, so its result does not depend
// on the rest of the batch.  Partials take up to 8 MiB per problem.
constexpr int64_t kSplitTiles = 128;
constexpr int64_t kSplitChunk = 256;
constexpr int64_t kPartDoubles = (kSplitTiles + kSplitTiles - 2) * kBatchTile * kBatchTile;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t even_up(int64_t v) { return (v + 1) & ~int64_t(1); }

struct Prob {
  // sizes
  int64_t m, n, kcap, ldr, ldm, ldc;
  int b;
  // device buffers
  double *R, *omega, *Y, *Qt, *Qi, *C, *G, *Tinv, *sqA, *sqB, *sqR, *part;
  int *flA, *kept;
  double* scal;  // [0..1] ||R||^2, [2..3] ||B_i||^2, [4..5] ||A||^2
  int* iflag;
  int64_t nconv;
};

bool problem_ok(const qb_problem& p) {
  if (!p.A || !p.Q || !p.B || p.m < 1 || p.n < 1 || p.b < 1 || p.b > kBMax) return false;
  if (!(p.eps >= 0.0) || !std::isfinite(p.eps)) return false;
  const int64_t r = std::min(p.m, p.n);
  const int64_t kcap = p.kmax < 0 ? r : p.kmax;
  if (kcap > r) return false;
  if (p.lda < p.m || p.ldq < p.m || p.ldb < std::max<int64_t>(kcap, 1)) return false;
  const int64_t lim = int64_t(1) << 24;  // 32-bit offsets inside a 64-row tile
  return p.lda < lim && p.ldq < lim && p.ldb < lim && p.m < lim && p.n < lim;
}

// device workspace: per-problem buffers, the scalar and kept tables, and one
// iteration's descriptors
constexpr int kSteps = 13;  // product steps of one block iteration

// static per-problem record (uploaded once per call)
struct DevProb {
  double *R, *omega, *Y, *Qt, *Qi, *C, *G, *Tinv, *sqB, *sqR, *part;
  int* kept;
  double* scal;
  int* iflag;
  double *Q, *B;
  int64_t m, n, kcap, ldr, ldm, ldc, ldq, ldb;
  uint64_t seed;
  double eps;
  int32_t b, pad;
};
// per-problem state across iterations
struct DevState {
  int64_t k;
  int32_t w, active, blocks, reason, status, pad;
  double sA_hi, sA_lo, sigB_hi, sigB_lo, eps2, delta, floor2, lastE, lastD;
};
struct TileTable {
  int32_t cls[QB_ROLES][3];
};

// device tables of one iteration
struct Plan {
  BatchGemm* gemm;      // [kSteps][kTileClasses][count]
  BatchGemm* rgemm;     // [kSteps][count] each problem's own entry, for the reduction
  int64_t* tiles;       // [kSteps][kTileClasses] units of each product launch
  int64_t* rblocks;     // [kSteps] units of each reduction launch
  int64_t* sk_blocks;   // [1] sketch units
  unsigned long long* next;  // [kSteps][kTileClasses] then [kSteps]: unit counters of the launches
  BatchSketch* sketch;  // [count]
  BatchChol *c1, *c3;   // [count] Cholesky of the first pair of passes / of the re-projected pair
  BatchSum *sB, *sR;    // [count]
  int* any_active;      // [1]
};

struct Layout {
  std::vector<Prob> pr;
  double* scal_all;
  int* kept_all;
  int* iflag_all;
  char* desc;       // device descriptor block
  size_t desc_bytes;
  DevProb* dprob;   // device-planned loop: static records, state, plan tables
  DevState* dstate;
  Plan plan;
};

size_t desc_block_bytes(int count) {
  return static_cast<size_t>(count) *
             (sizeof(BatchConvert) + sizeof(BatchSketch) + 14 * sizeof(BatchGemm) +
              4 * sizeof(BatchChol) + 3 * sizeof(BatchSum)) +
         64 * 32;
}

int carve_batch(Arena& a, const qb_problem* probs, int count, Layout* L) {
  L->pr.assign(count, Prob{});
  L->scal_all = a.take<double>(static_cast<size_t>(count) * kScal);
  L->kept_all = a.take<int>(static_cast<size_t>(count) * kKeptStride);
  L->iflag_all = a.take<int>(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    const qb_problem& q = probs[i];
    Prob& p = L->pr[i];
    const int64_t r = std::min(q.m, q.n);
    p.m = q.m;
    p.n = q.n;
    p.b = static_cast<int>(std::min<int64_t>(q.b, r));
    p.kcap = q.kmax < 0 ? r : q.kmax;
    p.ldr = even_up(q.m);
    p.ldm = even_up(q.m);
    p.ldc = std::max<int64_t>(p.kcap, 1);
    p.R = a.take<double>(static_cast<size_t>(p.ldr) * q.n);
    p.omega = a.take<double>(static_cast<size_t>(q.n) * p.b);
    p.Y = a.take<double>(static_cast<size_t>(p.ldm) * p.b);
    p.Qt = a.take<double>(static_cast<size_t>(p.ldm) * p.b);
    p.Qi = a.take<double>(static_cast<size_t>(p.ldm) * p.b);
    p.C = a.take<double>(static_cast<size_t>(p.ldc) * p.b);
    p.G = a.take<double>(static_cast<size_t>(p.b) * p.b);
    p.Tinv = a.take<double>(static_cast<size_t>(p.b) * p.b);
    p.nconv = convert_blocks(q.m, q.n);
    p.sqA = a.take<double>(static_cast<size_t>(p.nconv));
    p.flA = a.take<int>(static_cast<size_t>(p.nconv));
    // per-tile sums of squares of B_i and of the downdate, for tiles of at
    // least 32 x 32 (or per reduction workgroup of a split B_i)
    p.sqB = a.take<double>(static_cast<size_t>(std::max(cdiv(p.b, 32) * cdiv(q.n, 32),
                                                        cdiv(int64_t(p.b) * q.n, kBatchRed))));
    p.part = a.take<double>(static_cast<size_t>(kPartDoubles));
    p.sqR = a.take<double>(static_cast<size_t>(cdiv(q.m, 32) * cdiv(q.n, 32)));
    if (a.base != nullptr) {
      p.scal = L->scal_all + static_cast<size_t>(i) * kScal;
      p.kept = L->kept_all + static_cast<size_t>(i) * kKeptStride;
      p.iflag = L->iflag_all + i;
    }
  }
  L->desc_bytes = desc_block_bytes(count);
  L->desc = a.take<char>(L->desc_bytes);
  L->dprob = a.take<DevProb>(static_cast<size_t>(count));
  L->dstate = a.take<DevState>(static_cast<size_t>(count));
  Plan& pl = L->plan;
  pl.gemm = a.take<BatchGemm>(static_cast<size_t>(kSteps) * kTileClasses * count);
  pl.rgemm = a.take<BatchGemm>(static_cast<size_t>(kSteps) * count);
  pl.tiles = a.take<int64_t>(kSteps * kTileClasses);
  pl.rblocks = a.take<int64_t>(kSteps);
  pl.sk_blocks = a.take<int64_t>(1);
  pl.next = a.take<unsigned long long>(kSteps * kTileClasses + kSteps);
  pl.sketch = a.take<BatchSketch>(static_cast<size_t>(count));
  pl.c1 = a.take<BatchChol>(static_cast<size_t>(count));
  pl.c3 = a.take<BatchChol>(static_cast<size_t>(count));
  pl.sB = a.take<BatchSum>(static_cast<size_t>(count));
  pl.sR = a.take<BatchSum>(static_cast<size_t>(count));
  pl.any_active = a.take<int>(1);
  return (a.base != nullptr && a.used > a.cap) ? kEWorkspace : kOk;
}

// Per-thread pinned host memory for the descriptors and the per-iteration
// scalars, grown on demand and kept for the life of the thread (so a call
// allocates nothing once the thread has run a batch as large).  A call has
// synchronised its stream before returning, so the next one may reuse it.
void* pinned_stage(size_t bytes) {
  struct Pinned {
    void* p = nullptr;
    size_t cap = 0;
  };
  thread_local Pinned ps;
  if (bytes > ps.cap) {
    if (ps.p != nullptr) (void)hipHostFree(ps.p);
    ps.p = nullptr;
    ps.cap = 0;
    const size_t want = std::max(bytes + bytes / 4, size_t(1) << 20);
    if (hipHostMalloc(&ps.p, want, hipHostMallocDefault) != hipSuccess) {
      ps.p = nullptr;
      return nullptr;
    }
    ps.cap = want;
  }
  return ps.p;
}

// host staging of one iteration's descriptors; offsets into the device block
struct Stage {
  char* host = nullptr;
  size_t used = 0, cap = 0;
  bool overflow = false;
  template <class T>
  size_t put(const std::vector<T>& v) {
    used = (used + 63) & ~size_t(63);
    const size_t off = used;
    if (off + v.size() * sizeof(T) > cap) {
      overflow = true;
      return 0;
    }
    std::memcpy(host + off, v.data(), v.size() * sizeof(T));
    used += v.size() * sizeof(T);
    return off;
  }
};

// Tile class of each product role by panel width (w <= 16, <= 32, <= 64).
// The defaults are the table the tuner in autotune.py chose on every fourth
// problem of the 512-problem uneven workload (65 trials; the whole batch
// 230 -> 225 ms against the hand-picked table of k_gemm_batched.hip); they
// can be changed at run time through qb_batched_set_tile.  Every class
// computes the same products; the classes allowed for B_i and the downdate
// are those their per-tile sums of squares have room for.  Panels of 33..64
// columns keep 64 x 32 tiles for the samples, although two column tiles
// read R twice (counters: 1.8x the sample's algorithmic bytes at the first
// iteration): 64 x 64 tiles there read it once but made the batch 8 ms
// slower (half the workgroups, and one launch more per step).
std::atomic<int> g_tile[QB_ROLES][3] = {
    {{kTileN32}, {kTileN32}, {kTileN32}},  // QB_ROLE_SAMPLE     R Omega
    {{kTileG32}, {kTileG32}, {kTileG32}},  // QB_ROLE_GRAM       X^T X
    {{kTileN32}, {kTileN32}, {kTileN32}},  // QB_ROLE_APPLY      X T^{-1}
    {{kTileN32}, {kTileN32}, {kTileN32}},  // QB_ROLE_REPROJ_C   Qbar^T Q_i
    {{kTileN32}, {kTileN32}, {kTileG32}},  // QB_ROLE_REPROJ_Q   Q_i - Qbar C
    {{kTileM32}, {kTileM32}, {kTile64}},   // QB_ROLE_B          Q_i^T R
    {{kTile64}, {kTile64}, {kTile64}},     // QB_ROLE_DOWNDATE   R - Q_i B_i
};

int width_class(int w) { return w <= 16 ? 0 : w <= 32 ? 1 : 2; }
int tile_of(int role, int w) { return g_tile[role][width_class(w)].load(std::memory_order_relaxed); }

bool tile_allowed(int role, int wclass, int cls) {
  (void)wclass;
  if (cls < 0 || cls >= kTileClasses) return false;
  // B_i and the downdate leave one sum of squares per tile; their buffers
  // hold one per 32 x 32 tile
  if (role == QB_ROLE_B || role == QB_ROLE_DOWNDATE) return cls != kTileG16;
  return true;
}

// part: the problem's split-K buffer (kPartDoubles), or null for no split.
// Host and device (the device-planned loop) build the same descriptors.
__host__ __device__ BatchGemm gemm_desc(int cls, const double* A, int64_t lda, const double* B,
                                        int64_t ldb, double* C, int64_t ldc, int64_t M, int64_t N,
                                        int64_t K, double alpha, double beta, double* sq,
                                        double* part) {
  BatchGemm g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.sq = sq;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.M = static_cast<int32_t>(M);
  g.N = static_cast<int32_t>(N);
  g.K = static_cast<int32_t>(K);
  int bm = kBatchTile, bn = kBatchTile;
  batch_tile_dims_hd(cls, &bm, &bn);
  g.cls = cls;
  g.bm = bm;
  g.bn = bn;
  g.tiles_m = static_cast<int32_t>(cdiv(M, bm));
  g.tiles_n = static_cast<int32_t>(cdiv(N, bn));
  const bool va = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda & 1) == 0;
  const bool vb = (reinterpret_cast<uintptr_t>(B) & 15) == 0 && (ldb & 1) == 0;
  g.vec = (va && vb) ? 1 : 0;
  g.alpha = alpha;
  g.beta = beta;
  g.ksplit = 1;
  g.kchunk = static_cast<int32_t>(K);
  g.part = nullptr;
  const int64_t tiles = static_cast<int64_t>(g.tiles_m) * g.tiles_n;
  if (part != nullptr && tiles < kSplitTiles && K >= 2 * kSplitChunk) {
    int64_t ks = cdiv(kSplitTiles, tiles) < K / kSplitChunk ? cdiv(kSplitTiles, tiles)
                                                             : K / kSplitChunk;
    const int64_t chunk = cdiv(cdiv(K, ks), kTileK) * kTileK;
    ks = cdiv(K, chunk);
    if (ks > 1 && ks * tiles * bm * bn <= kPartDoubles) {
      g.ksplit = static_cast<int32_t>(ks);
      g.kchunk = static_cast<int32_t>(chunk);
      g.part = part;
    }
  }
  return g;
}

__host__ __device__ int64_t reduce_blocks(const BatchGemm& g) {
  return g.ksplit > 1 ? cdiv(static_cast<int64_t>(g.M) * g.N, kBatchRed) : 0;
}

// One step's product over the active problems, grouped by tile class: one
// launch per non-empty class (workgroup offsets tile0 within it), one
// reduction launch over all (offsets rblock0).
struct Step {
  std::vector<BatchGemm> d;
  int begin[kTileClasses + 1] = {};
  int64_t tiles[kTileClasses] = {};
  double flops[kTileClasses] = {};
  double bytes[kTileClasses] = {};
  int64_t rblocks = 0;
  size_t off = 0;
  int count() const { return static_cast<int>(d.size()); }
};

// reads_c: the product also reads C (the downdate, Qi -= Qbar C)
Step group(const std::vector<BatchGemm>& v, bool reads_c = false) {
  Step st;
  st.d.reserve(v.size());
  for (int c = 0; c < kTileClasses; ++c) {
    st.begin[c] = st.count();
    int64_t t = 0;
    for (const BatchGemm& g : v) {
      if (g.cls != c) continue;
      BatchGemm h = g;
      h.tile0 = t;
      t += static_cast<int64_t>(h.tiles_m) * h.tiles_n * h.ksplit;
      h.rblock0 = st.rblocks;
      st.rblocks += reduce_blocks(h);
      st.flops[c] += 2.0 * h.M * h.N * h.K;
      st.bytes[c] += 8.0 * (double(h.M) * h.K + double(h.K) * h.N +
                            double(h.M) * h.N * (reads_c ? 2.0 : 1.0));
      st.d.push_back(h);
    }
    st.tiles[c] = t;
  }
  st.begin[kTileClasses] = st.count();
  return st;
}

// partial sums of squares that a TN product with sq leaves per problem
__host__ __device__ int32_t sq_count(const BatchGemm& g) {
  return static_cast<int32_t>(g.ksplit > 1 ? reduce_blocks(g)
                                           : static_cast<int64_t>(g.tiles_m) * g.tiles_n);
}


// ---- device-planned block loop ---------------------------------------------
// The block loop's decisions (width, re-projection or not, the stopping rule)
// live on the device: a plan kernel writes every step's descriptors from the
// problems' state at the start of an iteration, the products walk the units
// the plan counted, and a stop kernel applies the rule of qb_factor to each
// problem.  Every launch of an iteration then has the same arguments, so the
// iterations are captured once in a HIP graph and replayed; the host reads
// one flag per replay (any problem still active).


// the steps of one iteration (product launches), in issue order
enum { kStY = 0, kStG1, kStA1, kStG2, kStA2, kStRC, kStRQ, kStG3, kStA3, kStG4, kStA4, kStB, kStD };
__host__ __device__ inline int step_op(int s) {
  return (s == kStG1 || s == kStG2 || s == kStRC || s == kStG3 || s == kStG4 || s == kStB)
             ? kBatchTN
             : (s == kStD ? kBatchDD : kBatchNN);
}
__host__ __device__ inline int step_role(int s) {
  switch (s) {
    case kStY: return QB_ROLE_SAMPLE;
    case kStG1: case kStG2: case kStG3: case kStG4: return QB_ROLE_GRAM;
    case kStA1: case kStA2: case kStA3: case kStA4: return QB_ROLE_APPLY;
    case kStRC: return QB_ROLE_REPROJ_C;
    case kStRQ: return QB_ROLE_REPROJ_Q;
    case kStB: return QB_ROLE_B;
    default: return QB_ROLE_DOWNDATE;
  }
}
__host__ __device__ inline int width_class_hd(int w) { return w <= 16 ? 0 : w <= 32 ? 1 : 2; }

// The descriptor of step s for problem p at width w and rank k (the same
// operands and pointers as the host-planned loop); false when p takes no
// part in the step.
__host__ __device__ bool step_desc(int s, const DevProb& p, int64_t k, int w, const TileTable& tt,
                          BatchGemm* g) {
  const int cls = tt.cls[step_role(s)][width_class_hd(w)];
  const bool rp = k > 0;  // re-projection steps run once a basis exists
  double* Qo = p.Q + k * p.ldq;
  switch (s) {
    case kStY:
      *g = gemm_desc(cls, p.R, p.ldr, p.omega, p.n, p.Y, p.ldm, p.m, w, p.n, 1.0, 0.0, nullptr, p.part);
      return true;
    case kStG1:
      *g = gemm_desc(cls, p.Y, p.ldm, p.Y, p.ldm, p.G, w, w, w, p.m, 1.0, 0.0, nullptr, p.part);
      return true;
    case kStA1:
      *g = gemm_desc(cls, p.Y, p.ldm, p.Tinv, w, p.Qt, p.ldm, p.m, w, w, 1.0, 0.0, nullptr, p.part);
      return true;
    case kStG2:
      *g = gemm_desc(cls, p.Qt, p.ldm, p.Qt, p.ldm, p.G, w, w, w, p.m, 1.0, 0.0, nullptr, p.part);
      return true;
    case kStA2:
      *g = gemm_desc(cls, p.Qt, p.ldm, p.Tinv, w, rp ? p.Qi : Qo, rp ? p.ldm : p.ldq, p.m, w, w,
                     1.0, 0.0, nullptr, p.part);
      return true;
    case kStRC:
      *g = gemm_desc(cls, p.Q, p.ldq, p.Qi, p.ldm, p.C, p.ldc, k, w, p.m, 1.0, 0.0, nullptr, p.part);
      return rp;
    case kStRQ:
      *g = gemm_desc(cls, p.Q, p.ldq, p.C, p.ldc, p.Qi, p.ldm, p.m, w, k, -1.0, 1.0, nullptr, p.part);
      return rp;
    case kStG3:
      *g = gemm_desc(cls, p.Qi, p.ldm, p.Qi, p.ldm, p.G, w, w, w, p.m, 1.0, 0.0, nullptr, p.part);
      return rp;
    case kStA3:
      *g = gemm_desc(cls, p.Qi, p.ldm, p.Tinv, w, p.Qt, p.ldm, p.m, w, w, 1.0, 0.0, nullptr, p.part);
      return rp;
    case kStG4:
      *g = gemm_desc(cls, p.Qt, p.ldm, p.Qt, p.ldm, p.G, w, w, w, p.m, 1.0, 0.0, nullptr, p.part);
      return rp;
    case kStA4:
      *g = gemm_desc(cls, p.Qt, p.ldm, p.Tinv, w, Qo, p.ldq, p.m, w, w, 1.0, 0.0, nullptr, p.part);
      return rp;
    case kStB:
      *g = gemm_desc(cls, Qo, p.ldq, p.R, p.ldr, p.B + k, p.ldb, w, p.n, p.m, 1.0, 0.0, p.sqB,
                     p.part);
      return true;
    default:
      *g = gemm_desc(cls, Qo, p.ldq, p.B + k, p.ldb, p.R, p.ldr, p.m, p.n, w, 1.0, 0.0, p.sqR,
                     nullptr);
      return true;
  }
}


constexpr int kPlanThreads = 256;

// exclusive scan of v over the workgroup (kPlanThreads); *total gets the sum
__device__ int64_t block_scan(int64_t v, int64_t* total, int64_t* buf) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  __syncthreads();
  if (lane == 63) buf[wave] = x;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kPlanThreads / 64; ++q) {
    if (q < wave) before += buf[q];
    all += buf[q];
  }
  *total = all;
  return before + x - v;
}

// workgroup s kTileClasses + c (s < kSteps): the descriptors of product
// step s in tile class c, with each problem's first unit (tile0), and the
// step's reduction descriptors (each problem's own entry, first reduction
// unit rblock0 in problem order; written by the workgroup of that problem's
// class, or of class 0 for a problem with none); workgroup kSteps
// kTileClasses: sketch, Cholesky and sum records
__global__ __launch_bounds__(kPlanThreads) void batch_plan_kernel(const DevProb* __restrict__ P,
                                                                  const DevState* __restrict__ S,
                                                                  int count, TileTable tt, Plan pl) {
  __shared__ int64_t buf[kPlanThreads / 64];
  const int wg = blockIdx.x;
  if (wg < kSteps * kTileClasses) {
    const int s = wg / kTileClasses, c = wg % kTileClasses;
    if (threadIdx.x == 0) pl.next[wg] = 0;
    if (c == 0 && threadIdx.x == 1) pl.next[kSteps * kTileClasses + s] = 0;
    BatchGemm* out = pl.gemm + static_cast<int64_t>(wg) * count;
    BatchGemm* rout = pl.rgemm + static_cast<int64_t>(s) * count;
    int64_t carry = 0, rcarry = 0;
    for (int i0 = 0; i0 < count; i0 += kPlanThreads) {
      const int i = i0 + static_cast<int>(threadIdx.x);
      BatchGemm g{};
      int64_t units = 0, runits = 0;
      int cls = -1;
      if (i < count && S[i].active) {
        const int w = S[i].w;
        if (step_desc(s, P[i], S[i].k, w, tt, &g)) {
          cls = tt.cls[step_role(s)][width_class_hd(w)];
          // a split Gram matrix is summed by the Cholesky that reads it
          runits = step_role(s) == QB_ROLE_GRAM ? 0 : reduce_blocks(g);
          if (cls == c) units = static_cast<int64_t>(g.tiles_m) * g.tiles_n * g.ksplit;
        }
      }
      int64_t tot = 0, rtot = 0;
      const int64_t ex = block_scan(units, &tot, buf);
      const int64_t rex = block_scan(runits, &rtot, buf);
      if (i < count) {
        if (cls != c) {  // no part in this launch: no units, no partial sums
          out[i] = BatchGemm{};
          out[i].ksplit = 1;
          out[i].tile0 = carry + ex;
        } else {
          g.tile0 = carry + ex;
          out[i] = g;
        }
        if (cls == c || (cls < 0 && c == 0)) {
          BatchGemm r = cls < 0 ? BatchGemm{} : g;
          if (cls < 0) r.ksplit = 1;
          r.rblock0 = rcarry + rex;
          rout[i] = r;
        }
      }
      carry += tot;
      rcarry += rtot;
    }
    if (threadIdx.x == 0) {
      pl.tiles[wg] = carry;
      if (c == 0) pl.rblocks[s] = rcarry;
    }
    return;
  }
  int64_t carry = 0;
  for (int i0 = 0; i0 < count; i0 += kPlanThreads) {
    const int i = i0 + static_cast<int>(threadIdx.x);
    int64_t units = 0;
    BatchSketch sk{};
    BatchChol c1{}, c3{};
    BatchSum sb{}, sr{};
    if (i < count && S[i].active) {
      const DevProb& p = P[i];
      const int w = S[i].w;
      const int64_t k = S[i].k;
      units = ((p.n + 1) / 2 + 255) / 256 * w;  // as sketch_blocks(n, w)
      sk = BatchSketch{p.seed, p.n, k, p.n, p.omega, 0, w};
      // the four Gram matrices of the iteration share one shape (w x w,
      // depth m) and so one depth split: the Cholesky sums their chunks
      BatchGemm gg;
      step_desc(kStG1, p, k, w, tt, &gg);
      const int64_t ldp = static_cast<int64_t>(gg.tiles_m) * gg.bm;
      c1 = BatchChol{p.G, p.kept, p.Tinv, w, gg.ksplit, gg.ksplit > 1 ? gg.part : nullptr, ldp,
                     ldp * (static_cast<int64_t>(gg.tiles_n) * gg.bn)};
      if (k > 0) c3 = c1;
      BatchGemm gb, gd;
      step_desc(kStB, p, k, w, tt, &gb);
      step_desc(kStD, p, k, w, tt, &gd);
      sb = BatchSum{p.sqB, nullptr, p.scal + 2, nullptr, sq_count(gb)};
      sr = BatchSum{p.sqR, nullptr, p.scal + 0, nullptr, sq_count(gd)};
    }
    int64_t tot = 0;
    const int64_t ex = block_scan(units, &tot, buf);
    if (i < count) {
      sk.block0 = carry + ex;
      pl.sketch[i] = sk;
      pl.c1[i] = c1;
      pl.c3[i] = c3;
      pl.sB[i] = sb;
      pl.sR[i] = sr;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *pl.sk_blocks = carry;
    *pl.any_active = 0;
  }
}

__device__ inline void dd_add_dev(double& hi, double& lo, double bh, double bl) {
  double s = hi + bh, bb = s - hi;
  double e = (hi - (s - bb)) + (bh - bb);
  e += lo + bl;
  const double s2 = s + e, bb2 = s2 - s;
  lo = (s - (s2 - bb2)) + (e - bb2);
  hi = s2;
}

__device__ inline void next_width(const DevProb& p, DevState& st) {
  const int64_t left = p.kcap - st.k;
  st.w = static_cast<int32_t>(left < p.b ? left : p.b);
  if (st.w <= 0) {
    st.active = 0;
    const int64_t r = p.m < p.n ? p.m : p.n;
    st.reason = p.kcap < r ? QB_STOP_KMAX : QB_STOP_RANK_CAP;
  }
}

// ||A||^2 and the non-finite flag of each problem -> the initial state
__global__ __launch_bounds__(256) void batch_init_kernel(const DevProb* __restrict__ P,
                                                         DevState* __restrict__ S, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const DevProb& p = P[i];
  DevState st{};
  st.reason = QB_STOP_ZERO;
  st.status = QB_OK;
  if (p.iflag[0]) {
    st.status = QB_ENONFINITE;
  } else {
    st.sA_hi = p.scal[4];
    st.sA_lo = p.scal[5];
    const double sAv = st.sA_hi + st.sA_lo;
    st.lastE = st.lastD = sAv;
    if (!isfinite(sAv)) {
      st.status = QB_EINVAL;
    } else {
      st.eps2 = p.eps * p.eps;
      st.delta = kDeltaRelB * sAv;
      const double f = kFloorRelB * sqrt(sAv);
      st.floor2 = f * f;
      st.active = sAv > st.eps2 ? 1 : 0;
      if (st.active) next_width(p, st);
    }
  }
  S[i] = st;
}

// the stopping rule of qb_factor after an iteration, per active problem
__global__ __launch_bounds__(256) void batch_stop_kernel(const DevProb* __restrict__ P,
                                                         DevState* __restrict__ S, int count,
                                                         int* __restrict__ any_active) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  DevState st = S[i];
  if (!st.active) return;
  const DevProb& p = P[i];
  const int wkept = p.kept[0];
  if (wkept <= 0) {
    st.active = 0;
    st.reason = QB_STOP_EXHAUSTED;
  } else {
    st.k += wkept;
    ++st.blocks;
    dd_add_dev(st.sigB_hi, st.sigB_lo, p.scal[2], p.scal[3]);
    double eh = st.sA_hi, el = st.sA_lo;
    dd_add_dev(eh, el, -st.sigB_hi, -st.sigB_lo);
    st.lastE = eh + el;
    st.lastD = p.scal[0] + p.scal[1];
    if (st.lastE <= st.eps2 - st.delta) {
      st.active = 0;
      st.reason = QB_STOP_TOL_TRACKED;
    } else if (!(st.lastE > st.eps2 + st.delta) && st.lastD <= st.eps2) {
      st.active = 0;
      st.reason = QB_STOP_TOL_DIRECT;
    } else if (st.lastD <= st.floor2) {
      st.active = 0;
      st.reason = QB_STOP_EXHAUSTED;
    } else {
      next_width(p, st);
    }
  }
  S[i] = st;
  if (st.active) atomicOr(any_active, 1);
}


}  // namespace
}  // namespace qb

using namespace qb;

extern "C" {

int qb_batched_set_tile(int32_t role, int32_t width_class, int32_t tile_class) {
  if (role < 0 || role >= QB_ROLES || width_class < 0 || width_class > 2) return QB_EINVAL;
  if (!tile_allowed(role, width_class, tile_class)) return QB_EINVAL;
  g_tile[role][width_class].store(tile_class, std::memory_order_relaxed);
  return QB_OK;
}

int qb_batched_get_tile(int32_t role, int32_t width_class) {
  if (role < 0 || role >= QB_ROLES || width_class < 0 || width_class > 2) return QB_EINVAL;
  return g_tile[role][width_class].load(std::memory_order_relaxed);
}

size_t qb_factor_batched_workspace_bytes(const qb_problem* probs, int32_t count) {
  if (!probs || count < 1) return 0;
  for (int i = 0; i < count; ++i)
    if (!problem_ok(probs[i])) return 0;
  Arena a{nullptr, 0, 0};
  Layout L;
  carve_batch(a, probs, count, &L);
  return a.used + 256;
}

int qb_factor_batched(qb_problem* probs, int32_t count, void* workspace, size_t ws_bytes,
                      void* stream) {
  Range rcall("qb_factor_batched");
  if (!probs || count < 1) return QB_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!problem_ok(probs[i])) return QB_EINVAL;
  if (workspace == nullptr) return QB_EWORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EINVAL;
  if (const int dv = device_ready()) return dv;
  Layout L;
  Arena arena{static_cast<char*>(workspace), ws_bytes, 0};
  if (carve_batch(arena, probs, count, &L) != kOk) return QB_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<Prob>& P = L.pr;

  // pinned host memory for the descriptors and the per-iteration scalars
  // (then the "still active" flag and two copies of the problems' state)
  Stage sg;
  sg.cap = L.desc_bytes;
  const size_t st_off = (sg.cap + 64 + 255) & ~size_t(255);
  const size_t st_bytes = static_cast<size_t>(count) * sizeof(DevState);
  void* hbuf = pinned_stage(st_off + 2 * st_bytes);
  if (hbuf == nullptr) return QB_EHIP;
  sg.host = static_cast<char*>(hbuf);
  int* hflag = reinterpret_cast<int*>(sg.host + sg.cap);  // the "still active" flag
  DevState* hstate2[2] = {reinterpret_cast<DevState*>(sg.host + st_off),
                          reinterpret_cast<DevState*>(sg.host + st_off + st_bytes)};
  auto upload = [&]() -> int {
    if (sg.used == 0) return kOk;
    return hipMemcpyAsync(L.desc, sg.host, sg.used, hipMemcpyHostToDevice, st) == hipSuccess
               ? kOk
               : kEHip;
  };
  auto dev = [&](size_t off) { return L.desc + off; };

  auto run = [&]() -> int {
    // ---- R = double(A), ||A||^2, non-finite check ----------------------
    {
      sg.used = 0;
      std::vector<BatchConvert> cv(count);
      std::vector<BatchSum> su(count);
      int64_t blocks = 0;
      for (int i = 0; i < count; ++i) {
        cv[i] = BatchConvert{probs[i].A, P[i].R, P[i].sqA, P[i].flA, probs[i].lda, P[i].ldr,
                             probs[i].m, probs[i].n, blocks};
        blocks += P[i].nconv;
        su[i] = BatchSum{P[i].sqA, P[i].flA, P[i].scal + 4, P[i].iflag,
                         static_cast<int32_t>(P[i].nconv)};
      }
      const size_t ocv = sg.put(cv), osu = sg.put(su);
      if (sg.overflow) return QB_EWORKSPACE;
      if (upload() || convert_batched(reinterpret_cast<BatchConvert*>(dev(ocv)), count, blocks, st) ||
          sum_batched(reinterpret_cast<BatchSum*>(dev(osu)), count, st))
        return QB_EHIP;
    }
    // ---- static records, initial state ---------------------------------
    {
      std::vector<DevProb> dp(count);
      for (int i = 0; i < count; ++i) {
        const Prob& p = P[i];
        const qb_problem& q = probs[i];
        dp[i] = DevProb{p.R, p.omega, p.Y, p.Qt, p.Qi, p.C, p.G, p.Tinv, p.sqB, p.sqR, p.part,
                        p.kept, p.scal, p.iflag, q.Q, q.B, p.m, p.n, p.kcap, p.ldr, p.ldm, p.ldc,
                        q.ldq, q.ldb, q.seed, q.eps, p.b, 0};
      }
      // appended after the conversion's descriptors: their copy to the
      // device may still be reading the staging buffer
      const size_t odp = sg.put(dp);
      if (sg.overflow) return QB_EWORKSPACE;
      if (hipMemcpyAsync(L.dprob, sg.host + odp, dp.size() * sizeof(DevProb),
                         hipMemcpyHostToDevice, st) != hipSuccess)
        return QB_EHIP;
      hipLaunchKernelGGL(batch_init_kernel, dim3(static_cast<unsigned>(cdiv(count, 256))), dim3(256),
                         0, st, L.dprob, L.dstate, count);
      if (hipGetLastError() != hipSuccess) return QB_EHIP;
    }

    // ---- launch plan: the classes each step may use and its grids --------
    TileTable tt;
    for (int r = 0; r < QB_ROLES; ++r)
      for (int c = 0; c < 3; ++c) tt.cls[r][c] = g_tile[r][c].load(std::memory_order_relaxed);
    // Grid of each launch: the units the problems that may still be active
    // could need at their widest (w = b, k = kcap), an upper bound on what
    // the device plans.  Recomputed (and the graph captured again) when the
    // problems left need less than half.
    int64_t grid[kSteps][kTileClasses] = {};
    int64_t rgrid[kSteps] = {};
    int64_t skgrid = 0;
    std::vector<char> alive(count, 1);
    // whether step st_ of problem p can ever split its depth (so needs the
    // reduction launch): gemm_desc splits only outputs of fewer than
    // kSplitTiles tiles with a depth of at least 2 kSplitChunk; the tile
    // count is smallest at w = 1 and k = 1, the depth fixed or growing
    auto may_split = [&](int st_, const Prob& p, const TileTable& t) {
      if (step_role(st_) == QB_ROLE_GRAM) return false;  // summed by the Cholesky
      for (int wc = 0; wc <= width_class_hd(p.b); ++wc) {
        int bm = 0, bn = 0;
        batch_tile_dims_hd(t.cls[step_role(st_)][wc], &bm, &bn);
        int64_t M = 1, N = 1, K = 0;
        switch (st_) {
          case kStY: M = p.m; K = p.n; break;
          case kStA1: case kStA2: case kStA3: case kStA4: M = p.m; K = p.b; break;
          case kStRC: K = p.m; break;
          case kStRQ: M = p.m; K = p.kcap; break;
          case kStB: N = p.n; K = p.m; break;
          default: K = p.m; break;  // the Gram matrices
        }
        if (cdiv(M, bm) * cdiv(N, bn) < kSplitTiles && K >= 2 * kSplitChunk) return true;
      }
      return false;
    };
    auto compute_grids = [&]() -> int64_t {
      for (auto& row : grid)
        for (int64_t& g : row) g = 0;
      for (int64_t& g : rgrid) g = 0;
      skgrid = 0;
      for (int i = 0; i < count; ++i) {
        if (!alive[i]) continue;
        const Prob& p = P[i];
        const int64_t w = p.b, k = p.kcap;
        skgrid += sketch_blocks(p.n, p.b);
        for (int st_ = 0; st_ < kSteps; ++st_) {
          int64_t M = 0, N = 0;
          switch (st_) {
            case kStY: case kStA1: case kStA2: case kStRQ: case kStA3: case kStA4: M = p.m; N = w; break;
            case kStRC: M = k; N = w; break;
            case kStB: M = w; N = p.n; break;
            case kStD: M = p.m; N = p.n; break;
            default: M = w; N = w; break;
          }
          bool seen[kTileClasses] = {};
          for (int wc = 0; wc <= width_class_hd(p.b); ++wc) {
            const int c = tt.cls[step_role(st_)][wc];
            if (seen[c]) continue;
            seen[c] = true;
            int bm = 0, bn = 0;
            batch_tile_dims_hd(c, &bm, &bn);
            grid[st_][c] += cdiv(M, bm) * cdiv(N, bn) + (st_ == kStD ? 0 : kSplitTiles);
          }
          // a reduction only where some width or rank could split the
          // product's depth: fewest tiles at w = 1 (k = 1 for Qbar^T Q_i)
          if (st_ != kStD && may_split(st_, p, tt)) rgrid[st_] += cdiv(M * N, kBatchRed);
        }
      }
      // workgroups launched per iteration with these grids
      int64_t tot = skgrid;
      for (int st_ = 0; st_ < kSteps; ++st_) {
        tot += rgrid[st_];
        for (int c = 0; c < kTileClasses; ++c) tot += grid[st_][c];
      }
      return tot;
    };
    int64_t grid_total = compute_grids();
    Plan pl = L.plan;
    const unsigned pgrid = static_cast<unsigned>(cdiv(count, 256));
    // eager: per-launch algorithmic work for the profiler from the host copy
    // of the state (read every iteration); graph: none
    std::vector<DevState> hs;
    auto issue = [&](hipStream_t cs, const DevState* hstate) -> int {
      hipLaunchKernelGGL(batch_plan_kernel, dim3(kSteps * kTileClasses + 1), dim3(kPlanThreads), 0,
                         cs, L.dprob, L.dstate, count, tt, pl);
      if (hipGetLastError() != hipSuccess) return 1;
      if (sketch_batched(pl.sketch, count, skgrid, cs, pl.sk_blocks)) return 1;
      auto mm = [&](int sidx, int pid) -> int {
        const int op = step_op(sidx);
        for (int c = 0; c < kTileClasses; ++c) {
          if (grid[sidx][c] == 0) continue;
          double fl = 0.0, by = 0.0;
          if (hstate) {
            for (int i = 0; i < count; ++i) {
              if (!hstate[i].active) continue;
              BatchGemm g;
              const DevProb pr{P[i].R, P[i].omega, P[i].Y, P[i].Qt, P[i].Qi, P[i].C, P[i].G,
                               P[i].Tinv, P[i].sqB, P[i].sqR, P[i].part, P[i].kept, P[i].scal,
                               P[i].iflag, probs[i].Q, probs[i].B, P[i].m, P[i].n, P[i].kcap,
                               P[i].ldr, P[i].ldm, P[i].ldc, probs[i].ldq, probs[i].ldb,
                               probs[i].seed, probs[i].eps, P[i].b, 0};
              if (!step_desc(sidx, pr, hstate[i].k, hstate[i].w, tt, &g) || g.cls != c) continue;
              fl += 2.0 * g.M * g.N * g.K;
              by += 8.0 * (double(g.M) * g.K + double(g.K) * g.N +
                           double(g.M) * g.N * ((op == kBatchDD || sidx == kStRQ) ? 2.0 : 1.0));
            }
          }
          const BatchGemm* d = pl.gemm + (static_cast<int64_t>(sidx) * kTileClasses + c) * count;
          if (gemm_batched(op, c, d, count, grid[sidx][c], pid, fl, by, cs,
                           pl.tiles + sidx * kTileClasses + c, pl.next + sidx * kTileClasses + c))
            return 1;
        }
        if (rgrid[sidx] == 0) return 0;
        return gemm_batched_reduce(op, pl.rgemm + static_cast<int64_t>(sidx) * count, count,
                                   rgrid[sidx], pid, cs,
                                   pl.rblocks + sidx, pl.next + kSteps * kTileClasses + sidx)
                   ? 1
                   : 0;
      };
      int e = 0;
      e = e || mm(kStY, kKBatchSample);
      e = e || mm(kStG1, kKBatchGram);
      e = e || chol_inv_batched(pl.c1, count, cs);
      e = e || mm(kStA1, kKBatchApply);
      e = e || mm(kStG2, kKBatchGram);
      e = e || chol_inv_batched(pl.c1, count, cs);
      e = e || mm(kStA2, kKBatchApply);
      e = e || mm(kStRC, kKBatchReproj);
      e = e || mm(kStRQ, kKBatchReproj);
      e = e || mm(kStG3, kKBatchGram);
      e = e || chol_inv_batched(pl.c3, count, cs);
      e = e || mm(kStA3, kKBatchApply);
      e = e || mm(kStG4, kKBatchGram);
      e = e || chol_inv_batched(pl.c3, count, cs);
      e = e || mm(kStA4, kKBatchApply);
      e = e || mm(kStB, kKBatchB);
      e = e || mm(kStD, kKBatchDowndate);
      e = e || sum_batched(pl.sB, count, cs);
      e = e || sum_batched(pl.sR, count, cs);
      if (e) return 1;
      hipLaunchKernelGGL(batch_stop_kernel, dim3(pgrid), dim3(256), 0, cs, L.dprob, L.dstate,
                         count, pl.any_active);
      return hipGetLastError() != hipSuccess ? 1 : 0;
    };
    auto more = [&]() -> int {  // 1: a problem is still active, 0: none, -1: error
      if (hipMemcpyAsync(hflag, pl.any_active, sizeof(int), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return -1;
      return hflag[0] != 0 ? 1 : 0;
    };

    // ---- block iterations ----------------------------------------------
    const bool eager = prof_enabled() || getenv("QB_BATCHED_EAGER") != nullptr;
    if (eager) {
      hs.resize(count);
      for (;;) {
        if (hipMemcpyAsync(hs.data(), L.dstate, count * sizeof(DevState), hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return QB_EHIP;
        if (issue(st, hs.data())) return QB_EHIP;
        // the one-workgroup-per-unit launches rely on the host grids
        // bounding the units the device planned: checked here, per
        // iteration (the graph path runs the same plan and bounds)
        int64_t ut[kSteps * kTileClasses], ur[kSteps], us = 0;
        if (hipMemcpyAsync(ut, pl.tiles, sizeof(ut), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(ur, pl.rblocks, sizeof(ur), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&us, pl.sk_blocks, sizeof(us), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return QB_EHIP;
        bool fits = us <= skgrid;
        for (int st_ = 0; st_ < kSteps; ++st_) {
          fits = fits && ur[st_] <= rgrid[st_];
          for (int c = 0; c < kTileClasses; ++c)
            fits = fits && ut[st_ * kTileClasses + c] <= grid[st_][c];
        }
        if (!fits) {
          std::fprintf(stderr, "qb_factor_batched: planned units exceed the launch grids\n");
          return QB_EHIP;
        }
        const int mo = more();
        if (mo < 0) return QB_EHIP;
        if (mo == 0) break;
      }
    } else {
      // kGraphIters iterations per graph; iterations after every problem
      // has stopped find nothing to do (empty plans).  Each replay is
      // enqueued before the host waits for the state after the previous
      // one, so the host's reading never leaves the GPU idle; the replay
      // enqueued after the last problem stopped runs empty.  Once the
      // problems left need less than half the captured grids, the graph is
      // captured again with grids for those problems only (the batch narrows
      // fast: a few long problems run the last half of the iterations
      // alone); the replaced graphs may still be running, so they are
      // destroyed at the end.
      constexpr int kGraphIters = 8;
      hipStream_t cs = nullptr;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      std::vector<std::pair<hipGraph_t, hipGraphExec_t>> retired;
      hipEvent_t ev[2] = {nullptr, nullptr};
      int e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess;
      for (hipEvent_t& x : ev)
        e = e || hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess;
      auto capture = [&]() -> int {
        if (exec || graph) retired.emplace_back(graph, exec);
        exec = nullptr;
        graph = nullptr;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return 1;
        int ce = 0;
        for (int u = 0; u < kGraphIters && !ce; ++u) ce = issue(cs, nullptr);
        const bool ended = hipStreamEndCapture(cs, &graph) == hipSuccess;
        if (ce || !ended) return 1;
        return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess;
      };
      // one replay and the copy of the state after it into hstate2[b]
      auto replay = [&](int b) -> int {
        return hipGraphLaunch(exec, st) != hipSuccess ||
               hipMemcpyAsync(hstate2[b], L.dstate, st_bytes, hipMemcpyDeviceToHost, st) !=
                   hipSuccess ||
               hipEventRecord(ev[b], st) != hipSuccess;
      };
      if (!e) e = capture();
      if (!e) e = replay(0);
      int cur = 0;
      while (!e) {
        Range rrep("qb_batched_graph_replay");
        if (replay(cur ^ 1) || hipEventSynchronize(ev[cur]) != hipSuccess) {
          e = 1;
          break;
        }
        const DevState* hsr = hstate2[cur];
        bool any = false;
        for (int i = 0; i < count; ++i) {
          alive[i] = hsr[i].active ? 1 : 0;
          any = any || hsr[i].active;
        }
        if (!any) break;
        int64_t old_grid[kSteps][kTileClasses], old_rgrid[kSteps], old_sk = skgrid;
        std::memcpy(old_grid, grid, sizeof(grid));
        std::memcpy(old_rgrid, rgrid, sizeof(rgrid));
        const int64_t need = compute_grids();
        if (2 * need < grid_total) {
          grid_total = need;
          e = capture();
        } else {  // keep the captured graph and its grids
          std::memcpy(grid, old_grid, sizeof(grid));
          std::memcpy(rgrid, old_rgrid, sizeof(rgrid));
          skgrid = old_sk;
        }
        cur ^= 1;
      }
      // every replay has finished before anything is destroyed
      if (hipStreamSynchronize(st) != hipSuccess) e = 1;
      for (auto& ge : retired) {
        if (ge.second) (void)hipGraphExecDestroy(ge.second);
        if (ge.first) (void)hipGraphDestroy(ge.first);
      }
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
      if (cs) (void)hipStreamDestroy(cs);
      if (e) return QB_EHIP;
    }

    // ---- outputs ---------------------------------------------------------
    hs.resize(count);
    if (hipMemcpyAsync(hs.data(), L.dstate, count * sizeof(DevState), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QB_EHIP;
    for (int i = 0; i < count; ++i) {
      qb_problem& q = probs[i];
      const DevState& d = hs[i];
      q.k = d.k;
      q.blocks = d.blocks;
      q.stop_reason = d.reason;
      q.normA2 = d.sA_hi + d.sA_lo;
      q.resid2 = d.lastD;
      if (d.status != QB_OK) {
        q.status = d.status;
        q.k = 0;
        q.blocks = 0;
        q.stop_reason = QB_STOP_ZERO;
        continue;
      }
      q.status = (d.reason == QB_STOP_ZERO || d.reason == QB_STOP_TOL_TRACKED ||
                  d.reason == QB_STOP_TOL_DIRECT)
                     ? QB_OK
                     : (d.reason == QB_STOP_KMAX ? QB_KMAX : QB_RANK_EXHAUSTED);
    }
    return QB_OK;
  };
  const int rc = run();
  // the staging buffer is reused by the thread's next call: nothing queued
  // may still read or write it (a failed run can leave copies in flight)
  if (rc != QB_OK) (void)hipStreamSynchronize(st);
  return rc;
}

}  // extern "C"
