// Batched blocked QB: many independent problems (Figure 4, P = 0) advanced
// together, one launch per step of the block loop for every active problem.
//
// Each block iteration runs, for all problems still active:
//   sketch -> Y = R Omega -> CholQR2 (Gram, Cholesky + inverse, apply) ->
//   [k > 0: C = Qbar^T Q, Q -= Qbar C, CholQR2] -> B_i = Q_i^T R with
//   ||B_i||^2 -> R -= Q_i B_i with ||R||^2 -> per-problem compensated sums,
// then copies every problem's scalars to the host at once and applies the
// same stopping rule as qb_factor to each.  Problems stop independently;
// the launches of an iteration cover only the active ones.  Products use
// MFMA tiles of a class chosen per product role and panel width (a table,
// see g_tile), one launch per class in use, with a workgroup -> (problem,
// tile, depth chunk) mapping; the Cholesky runs one workgroup per problem.
// Inputs are float; every stored value and every product is float64, so
// each problem follows the float64 oracle.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
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
// longest problem alone from 69 to 45 ms; 256 gave no further gain).  The
// choice depends only on the problem's own sizes, so its result does not
// depend on the rest of the batch.  Partials take up to 4 MiB per problem.
constexpr int64_t kSplitTiles = 64;
constexpr int64_t kSplitChunk = 256;
constexpr int64_t kPartDoubles = (kSplitTiles + kSplitTiles - 2) * kBatchTile * kBatchTile;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t even_up(int64_t v) { return (v + 1) & ~int64_t(1); }

struct DD {
  double hi, lo;
};
inline DD two_sum_h(double a, double b) {
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
inline DD dd_add(DD x, DD y) {
  DD s = two_sum_h(x.hi, y.hi);
  s.lo += x.lo + y.lo;
  return two_sum_h(s.hi, s.lo);
}

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
  // host state
  int64_t k = 0;
  int blocks = 0, reason = QB_STOP_ZERO, w = 0;
  bool active = false;
  DD sA{0, 0}, sigB{0, 0};
  double eps2 = 0, delta = 0, floor2 = 0, lastE = 0, lastD = 0;
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
struct Layout {
  std::vector<Prob> pr;
  double* scal_all;
  int* kept_all;
  int* iflag_all;
  char* desc;       // device descriptor block
  size_t desc_bytes;
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
// are those their per-tile sums of squares have room for.
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

// part: the problem's split-K buffer (kPartDoubles), or null for no split
BatchGemm gemm_desc(int cls, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C, int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha,
                    double beta, double* sq, double* part) {
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
  batch_tile_dims(cls, &bm, &bn);
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
    int64_t ks = std::min(cdiv(kSplitTiles, tiles), K / kSplitChunk);
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

int64_t reduce_blocks(const BatchGemm& g) {
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
int32_t sq_count(const BatchGemm& g) {
  return static_cast<int32_t>(g.ksplit > 1 ? reduce_blocks(g)
                                           : static_cast<int64_t>(g.tiles_m) * g.tiles_n);
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
  Stage sg;
  sg.cap = L.desc_bytes;
  const size_t scal_bytes = static_cast<size_t>(count) * kScal * sizeof(double);
  const size_t kept_bytes = static_cast<size_t>(count) * kKeptStride * sizeof(int);
  const size_t flag_bytes = static_cast<size_t>(count) * sizeof(int);
  void* hbuf = pinned_stage(sg.cap + scal_bytes + kept_bytes + flag_bytes);
  if (hbuf == nullptr) return QB_EHIP;
  sg.host = static_cast<char*>(hbuf);
  double* hscal = reinterpret_cast<double*>(sg.host + sg.cap);
  int* hkept = reinterpret_cast<int*>(sg.host + sg.cap + scal_bytes);
  int* hflag = reinterpret_cast<int*>(sg.host + sg.cap + scal_bytes + kept_bytes);
  auto upload = [&]() -> int {
    if (sg.used == 0) return kOk;
    return hipMemcpyAsync(L.desc, sg.host, sg.used, hipMemcpyHostToDevice, st) == hipSuccess
               ? kOk
               : kEHip;
  };
  auto dev = [&](size_t off) { return L.desc + off; };
  auto fetch = [&]() -> int {
    if (hipMemcpyAsync(hscal, L.scal_all, scal_bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hkept, L.kept_all, kept_bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hflag, L.iflag_all, flag_bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return kEHip;
    return kOk;
  };

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
          sum_batched(reinterpret_cast<BatchSum*>(dev(osu)), count, st) || fetch())
        return QB_EHIP;
    }
    for (int i = 0; i < count; ++i) {
      Prob& p = P[i];
      qb_problem& q = probs[i];
      q.k = 0;
      q.blocks = 0;
      q.stop_reason = QB_STOP_ZERO;
      if (hflag[i]) {
        q.status = QB_ENONFINITE;
        continue;
      }
      p.sA = DD{hscal[i * kScal + 4], hscal[i * kScal + 5]};
      const double sAv = p.sA.hi + p.sA.lo;
      q.normA2 = sAv;
      q.resid2 = sAv;
      if (!std::isfinite(sAv)) {
        q.status = QB_EINVAL;
        continue;
      }
      p.eps2 = q.eps * q.eps;
      p.delta = kDeltaRelB * sAv;
      p.floor2 = (kFloorRelB * std::sqrt(sAv)) * (kFloorRelB * std::sqrt(sAv));
      p.lastE = p.lastD = sAv;
      q.status = QB_OK;
      p.active = sAv > p.eps2;
    }

    // ---- block iterations ----------------------------------------------
    for (;;) {
      std::vector<int> act;
      for (int i = 0; i < count; ++i) {
        Prob& p = P[i];
        if (!p.active) continue;
        p.w = static_cast<int>(std::min<int64_t>(p.b, p.kcap - p.k));
        if (p.w <= 0) {
          p.active = false;
          p.reason = p.kcap < std::min(p.m, p.n) ? QB_STOP_KMAX : QB_STOP_RANK_CAP;
          continue;
        }
        act.push_back(i);
      }
      if (act.empty()) break;
      sg.used = 0;
      sg.overflow = false;
      const int na = static_cast<int>(act.size());
      // sketch
      std::vector<BatchSketch> sk(na);
      int64_t skb = 0;
      for (int a = 0; a < na; ++a) {
        const Prob& p = P[act[a]];
        sk[a] = BatchSketch{probs[act[a]].seed, p.n, p.k, p.n, p.omega, skb, p.w};
        skb += sketch_blocks(p.n, p.w);
      }
      // Y = R Omega
      std::vector<BatchGemm> gY(na);
      for (int a = 0; a < na; ++a) {
        const Prob& p = P[act[a]];
        gY[a] = gemm_desc(tile_of(QB_ROLE_SAMPLE, p.w), p.R, p.ldr, p.omega, p.n, p.Y, p.ldm, p.m, p.w, p.n, 1.0,
                          0.0, nullptr, p.part);
      }
      // CholQR pass helpers: Gram, Cholesky, apply into dst
      auto gram = [&](const std::vector<int>& ids, double* const* X) {
        std::vector<BatchGemm> g(ids.size());
        for (size_t a = 0; a < ids.size(); ++a) {
          const Prob& p = P[ids[a]];
          g[a] = gemm_desc(tile_of(QB_ROLE_GRAM, p.w), X[a], p.ldm, X[a], p.ldm, p.G, p.w, p.w, p.w, p.m, 1.0,
                           0.0, nullptr, p.part);
        }
        return g;
      };
      auto chol = [&](const std::vector<int>& ids) {
        std::vector<BatchChol> c(ids.size());
        for (size_t a = 0; a < ids.size(); ++a) {
          const Prob& p = P[ids[a]];
          c[a] = BatchChol{p.G, p.kept, p.Tinv, p.w};
        }
        return c;
      };
      auto apply = [&](const std::vector<int>& ids, double* const* X, double* const* D,
                       const int64_t* ldd) {
        std::vector<BatchGemm> g(ids.size());
        for (size_t a = 0; a < ids.size(); ++a) {
          const Prob& p = P[ids[a]];
          g[a] = gemm_desc(tile_of(QB_ROLE_APPLY, p.w), X[a], p.ldm, p.Tinv, p.w, D[a], ldd[a], p.m, p.w, p.w,
                           1.0, 0.0, nullptr, p.part);
        }
        return g;
      };
      std::vector<int> reproj;
      for (int a = 0; a < na; ++a)
        if (P[act[a]].k > 0) reproj.push_back(act[a]);
      const int nr = static_cast<int>(reproj.size());
      // pass 1 on Y -> Qt; pass 2 on Qt -> (k == 0 ? Q + k ldq : Qi)
      std::vector<double*> xY(na), xQt(na), dQt(na), d2(na);
      std::vector<int64_t> lQt(na), l2(na);
      for (int a = 0; a < na; ++a) {
        Prob& p = P[act[a]];
        qb_problem& q = probs[act[a]];
        xY[a] = p.Y;
        xQt[a] = p.Qt;
        dQt[a] = p.Qt;
        lQt[a] = p.ldm;
        d2[a] = p.k > 0 ? p.Qi : q.Q + p.k * q.ldq;
        l2[a] = p.k > 0 ? p.ldm : q.ldq;
      }
      std::vector<BatchGemm> g1 = gram(act, xY.data()), a1 = apply(act, xY.data(), dQt.data(), lQt.data());
      std::vector<BatchGemm> g2 = gram(act, xQt.data()), a2 = apply(act, xQt.data(), d2.data(), l2.data());
      std::vector<BatchChol> c1 = chol(act);

      // re-projection of the problems with k > 0, then CholQR2 into Q + k ldq
      std::vector<BatchGemm> rC(nr), rQ(nr);
      std::vector<double*> xQi(nr), dQt2(nr), xQt2(nr), dOut(nr);
      std::vector<int64_t> lQt2(nr), lOut(nr);
      for (int a = 0; a < nr; ++a) {
        Prob& p = P[reproj[a]];
        qb_problem& q = probs[reproj[a]];
        rC[a] = gemm_desc(tile_of(QB_ROLE_REPROJ_C, p.w), q.Q, q.ldq, p.Qi, p.ldm, p.C, p.ldc, p.k, p.w, p.m, 1.0,
                          0.0, nullptr, p.part);
        rQ[a] = gemm_desc(tile_of(QB_ROLE_REPROJ_Q, p.w), q.Q, q.ldq, p.C, p.ldc, p.Qi, p.ldm, p.m, p.w, p.k, -1.0,
                          1.0, nullptr, p.part);
        xQi[a] = p.Qi;
        dQt2[a] = p.Qt;
        xQt2[a] = p.Qt;
        lQt2[a] = p.ldm;
        dOut[a] = q.Q + p.k * q.ldq;
        lOut[a] = q.ldq;
      }
      std::vector<BatchGemm> g3 = gram(reproj, xQi.data()), a3 = apply(reproj, xQi.data(), dQt2.data(), lQt2.data());
      std::vector<BatchGemm> g4 = gram(reproj, xQt2.data()), a4 = apply(reproj, xQt2.data(), dOut.data(), lOut.data());
      std::vector<BatchChol> c3 = chol(reproj);

      // B_i = Q_i^T R with ||B_i||^2, R -= Q_i B_i with ||R||^2, sums
      std::vector<BatchGemm> gB(na), gD(na);
      std::vector<BatchSum> sB(na), sR(na);
      for (int a = 0; a < na; ++a) {
        Prob& p = P[act[a]];
        qb_problem& q = probs[act[a]];
        double* Qo = q.Q + p.k * q.ldq;
        double* Bo = q.B + p.k;
        gB[a] = gemm_desc(tile_of(QB_ROLE_B, p.w), Qo, q.ldq, p.R, p.ldr, Bo, q.ldb, p.w, p.n, p.m, 1.0, 0.0,
                          p.sqB, p.part);
        gD[a] = gemm_desc(tile_of(QB_ROLE_DOWNDATE, p.w), Qo, q.ldq, Bo, q.ldb, p.R, p.ldr, p.m, p.n, p.w, 1.0, 0.0,
                          p.sqR, nullptr);
        sB[a] = BatchSum{p.sqB, nullptr, p.scal + 2, nullptr, sq_count(gB[a])};
        sR[a] = BatchSum{p.sqR, nullptr, p.scal + 0, nullptr, sq_count(gD[a])};
      }


      Step sY = group(gY), s1 = group(g1), sa1 = group(a1), s2 = group(g2), sa2 = group(a2);
      Step srC = group(rC), srQ = group(rQ, true), s3 = group(g3), sa3 = group(a3),
           s4 = group(g4), sa4 = group(a4);
      Step sBB = group(gB), sDD = group(gD, true);
      const size_t osk = sg.put(sk);
      for (Step* x : {&sY, &s1, &sa1, &s2, &sa2}) x->off = sg.put(x->d);
      const size_t oc1 = sg.put(c1);
      size_t oc3 = 0;
      if (nr) {
        for (Step* x : {&srC, &srQ, &s3, &sa3, &s4, &sa4}) x->off = sg.put(x->d);
        oc3 = sg.put(c3);
      }
      sBB.off = sg.put(sBB.d);
      sDD.off = sg.put(sDD.d);
      const size_t osB = sg.put(sB), osR = sg.put(sR);
      if (sg.overflow) return QB_EWORKSPACE;
      auto G = [&](size_t off) { return reinterpret_cast<const BatchGemm*>(dev(off)); };
      auto Ch = [&](size_t off) { return reinterpret_cast<const BatchChol*>(dev(off)); };
      int e = upload();
      e = e || sketch_batched(reinterpret_cast<const BatchSketch*>(dev(osk)), na, skb, st);
      auto mm = [&](int op, const Step& x, int pid) -> int {
        for (int c = 0; c < kTileClasses; ++c) {
          const int cnt = x.begin[c + 1] - x.begin[c];
          if (cnt == 0) continue;
          if (gemm_batched(op, c, G(x.off) + x.begin[c], cnt, x.tiles[c], pid, x.flops[c],
                           x.bytes[c], st))
            return 1;
        }
        return gemm_batched_reduce(op, G(x.off), x.count(), x.rblocks, pid, st) ? 1 : 0;
      };
      e = e || mm(kBatchNN, sY, kKBatchSample);
      e = e || mm(kBatchTN, s1, kKBatchGram);
      e = e || chol_inv_batched(Ch(oc1), na, st);
      e = e || mm(kBatchNN, sa1, kKBatchApply);
      e = e || mm(kBatchTN, s2, kKBatchGram);
      e = e || chol_inv_batched(Ch(oc1), na, st);
      e = e || mm(kBatchNN, sa2, kKBatchApply);
      if (nr) {
        e = e || mm(kBatchTN, srC, kKBatchReproj);
        e = e || mm(kBatchNN, srQ, kKBatchReproj);
        e = e || mm(kBatchTN, s3, kKBatchGram);
        e = e || chol_inv_batched(Ch(oc3), nr, st);
        e = e || mm(kBatchNN, sa3, kKBatchApply);
        e = e || mm(kBatchTN, s4, kKBatchGram);
        e = e || chol_inv_batched(Ch(oc3), nr, st);
        e = e || mm(kBatchNN, sa4, kKBatchApply);
      }
      e = e || mm(kBatchTN, sBB, kKBatchB);
      e = e || mm(kBatchDD, sDD, kKBatchDowndate);
      e = e || sum_batched(reinterpret_cast<const BatchSum*>(dev(osB)), na, st);
      e = e || sum_batched(reinterpret_cast<const BatchSum*>(dev(osR)), na, st);
      e = e || fetch();
      if (e) return QB_EHIP;
      // the stopping rule of qb_factor, per problem
      for (int a = 0; a < na; ++a) {
        const int i = act[a];
        Prob& p = P[i];
        const int wkept = hkept[i * kKeptStride];
        if (wkept <= 0) {
          p.active = false;
          p.reason = QB_STOP_EXHAUSTED;
          continue;
        }
        p.k += wkept;
        ++p.blocks;
        p.sigB = dd_add(p.sigB, DD{hscal[i * kScal + 2], hscal[i * kScal + 3]});
        const DD Edd = dd_add(p.sA, DD{-p.sigB.hi, -p.sigB.lo});
        p.lastE = Edd.hi + Edd.lo;
        p.lastD = hscal[i * kScal + 0] + hscal[i * kScal + 1];
        if (p.lastE <= p.eps2 - p.delta) {
          p.active = false;
          p.reason = QB_STOP_TOL_TRACKED;
        } else if (!(p.lastE > p.eps2 + p.delta) && p.lastD <= p.eps2) {
          p.active = false;
          p.reason = QB_STOP_TOL_DIRECT;
        } else if (p.lastD <= p.floor2) {
          p.active = false;
          p.reason = QB_STOP_EXHAUSTED;
        } else if (p.k >= p.kcap) {
          p.active = false;
          p.reason = p.kcap < std::min(p.m, p.n) ? QB_STOP_KMAX : QB_STOP_RANK_CAP;
        }
      }
    }
    for (int i = 0; i < count; ++i) {
      qb_problem& q = probs[i];
      if (q.status != QB_OK) continue;
      const Prob& p = P[i];
      q.k = p.k;
      q.blocks = p.blocks;
      q.stop_reason = p.reason;
      q.resid2 = p.lastD;
      q.status = (p.reason == QB_STOP_ZERO || p.reason == QB_STOP_TOL_TRACKED ||
                  p.reason == QB_STOP_TOL_DIRECT)
                     ? QB_OK
                     : (p.reason == QB_STOP_KMAX ? QB_KMAX : QB_RANK_EXHAUSTED);
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
