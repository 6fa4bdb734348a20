// Batched FP64 MFMA products: every active problem's product of one step of
// the batched block loop in one launch.  Workgroup -> (problem, tile, depth
// chunk) by binary search over the problems' first workgroup indices; the
// tile loop and epilogues are those of the single-matrix kernels
// (gemm_tiles.hpp).  Problems whose product is split over depth chunks
// leave their partial tiles to gemm_batched_reduce, which sums them in chunk
// order, so results are bitwise reproducible.
#include <cstdlib>

#include "gemm_tiles.hpp"

namespace qb {
namespace {

// Tile choices, measured on 512 uneven problems (ms per batch):
//   * Gram matrices of panels w <= 16 or 32: 16 x 16 / 32 x 32 tiles, so
//     neither side of the MFMA work is padded to 64 (Gram 25 -> 21 ms);
//   * the other products of panels w <= 32 (R Omega, the T^{-1}
//     application, Qbar C, Qbar^T Q_i; Q_i^T R): 64 x 32 / 32 x 64 tiles of
//     four waves side by side along the long side, padding to 32 instead
//     of 64 (batch 249 -> 229..234 ms over runs).  Two-wave 32 x 16 / 16 x 32 tiles for
//     w <= 16 were slower (239 ms), as were 128 x 16 / 16 x 128 with two
//     waves and 256 x 64 for R Omega: these products are bound by each
//     workgroup's depth loop, and four-wave tiles with many workgroups win;
//   * the downdate, a stream over R: 64 x 64 (69 ms) against 32 x 32
//     (75 ms) and 128 x 128 (178 ms).
// (A workgroup-parallel search for the owning problem in place of the
// binary search below measured the same, 234 ms: not the bottleneck.)
using BatchG16 = Shape<16, 16, 1, 1>;
using BatchG32 = Shape<32, 32, 2, 2>;
// Panels w <= 32 wide: four waves side by side along the long side, so the
// narrow side is padded to 32 instead of 64 with the same number of waves.
using BatchN32 = Shape<64, 32, 4, 1>;
using BatchM32 = Shape<32, 64, 1, 4>;

// LDS of a batched product workgroup: the two operand stages, which the
// downdate reuses for its product tile (BN columns of BM + 2 doubles) once
// the depth loop is done.
template <class S>
struct BatchLds {
  static constexpr int kStage = 2 * S::A_LDS + 2 * S::B_LDS;
  static constexpr int kLdc = S::BM + 2;  // even: 16-byte pairs stay aligned
  static constexpr int kTile = S::BN * kLdc;
  static constexpr int kSize = kStage > kTile ? kStage : kTile;
};

// Downdate C -= A B of one tile (depth K = the panel width, one chunk).  The
// old tile is read, and the new one written, in 16-byte row pairs that run
// down each column (a wave moves whole 512- or 256-byte column segments);
// the product goes from the MFMA result layout (four rows of one column per
// lane) to that layout through LDS.  Reading C in the result layout instead
// split every 128-byte line over two load instructions and held the
// downdate to about 3.8 TB/s of traffic against 5.6 TB/s for a plain
// read-modify-write stream.  Returns the tile's sum of squares to thread 0.
__device__ __forceinline__ int left_in_tile(int64_t M, int64_t m0, int tile) {
  return M - m0 < tile ? static_cast<int>(M - m0) : tile;
}

template <class S>
__device__ __forceinline__ double downdate_tile(const BatchGemm& g, int64_t m0, int64_t n0,
                                                int64_t kbeg, int64_t kend, double* As,
                                                double* Bs, double* red) {
  constexpr int PR = S::BM / 2;                     // row pairs per column
  constexpr int CH = S::BM * S::BN / (2 * S::NT);  // pairs per thread
  constexpr int LDC = BatchLds<S>::kLdc;
  static_assert(CH * 2 * S::NT == S::BM * S::BN, "whole pairs per thread");
  // rows and columns left in the tile; element offsets from the tile origin
  // fit in 32 bits (batched dimensions and leading dimensions stay below
  // 2^24, checked when the call is validated)
  const int mv = left_in_tile(g.M, m0, S::BM), nv = left_in_tile(g.N, n0, S::BN);
  const uint32_t ldc = static_cast<uint32_t>(g.ldc);
  double* const base = g.C + m0 + n0 * g.ldc;
  const int tid = threadIdx.x;
  const bool vc = vec_ok_dev(g.C, g.ldc);
  double2 c[CH];
#pragma unroll
  for (int q = 0; q < CH; ++q) {  // issued before the depth loop: latency overlaps it
    const int id = tid + S::NT * q;
    const int col = id / PR, row = 2 * (id % PR);
    const double* p = base + (static_cast<uint32_t>(row) + static_cast<uint32_t>(col) * ldc);
    c[q] = make_double2(0.0, 0.0);
    if (col < nv) {
      if (vc && row + 1 < mv) {
        c[q] = *reinterpret_cast<const double2*>(p);
      } else {
        if (row < mv) c[q].x = p[0];
        if (row + 1 < mv) c[q].y = p[1];
      }
    }
  }
  d4 acc[S::IB][S::JB];
  // ends with a barrier after its last LDS read (or touches no LDS)
  mma_loop<S, false>(g.A, g.lda, g.B, g.ldb, m0, n0, g.M, g.N, kbeg, kend, g.vec != 0, As, Bs,
                     acc);
  double* L = As;
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      double* d = L + acc_col<S>(j) * LDC + acc_row0<S>(i);
      *reinterpret_cast<double2*>(d) = make_double2(acc[i][j][0], acc[i][j][1]);
      *reinterpret_cast<double2*>(d + 2) = make_double2(acc[i][j][2], acc[i][j][3]);
    }
  __syncthreads();
  double sq = 0.0;
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const int id = tid + S::NT * q;
    const int col = id / PR, row = 2 * (id % PR);
    const double2 a = *reinterpret_cast<const double2*>(L + col * LDC + row);
    const double2 v = make_double2(c[q].x - a.x, c[q].y - a.y);
    if (col < nv) {
      double* p = base + (static_cast<uint32_t>(row) + static_cast<uint32_t>(col) * ldc);
      if (vc && row + 1 < mv) {
        *reinterpret_cast<double2*>(p) = v;
        sq += v.x * v.x + v.y * v.y;
      } else {
        if (row < mv) {
          p[0] = v.x;
          sq += v.x * v.x;
        }
        if (row + 1 < mv) {
          p[1] = v.y;
          sq += v.y * v.y;
        }
      }
    }
  }
  return block_sum(sq, red);
}

// One (problem, tile, depth chunk) of a batched product: workgroup-uniform
// blk; the LDS stages are free again when it returns (the depth loop ends
// with a barrier, the epilogue's sum synchronises).
template <class S, int OP>
__device__ __forceinline__ void batched_tile(const BatchGemm* __restrict__ desc, int count,
                                             int64_t blk, double* As, double* Bs, double* red) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {  // last problem with tile0 <= blk
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  const BatchGemm g = desc[lo];
  const int64_t tiles = static_cast<int64_t>(g.tiles_m) * g.tiles_n;
  const int64_t u = blk - g.tile0;
  const int64_t kz = u / tiles, t = u - kz * tiles;
  const int64_t m0 = (t % g.tiles_m) * S::BM;
  const int64_t n0 = (t / g.tiles_m) * S::BN;
  const int64_t M = g.M, N = g.N, K = g.K;
  const int64_t kbeg = kz * g.kchunk;
  const int64_t kend = kbeg + g.kchunk < K ? kbeg + g.kchunk : K;
  if constexpr (OP == kBatchDD) {  // never split: the depth is the panel width
    const double tot = downdate_tile<S>(g, m0, n0, kbeg, kend, As, Bs, red);
    if (g.sq != nullptr && threadIdx.x == 0) g.sq[t] = tot;
    return;
  }
  const bool vc = vec_ok_dev(g.C, g.ldc);
  const bool need = g.ksplit == 1 && OP == kBatchNN && g.beta != 0.0;
  d4 acc[S::IB][S::JB];
  mma_loop<S, OP == kBatchTN>(g.A, g.lda, g.B, g.ldb, m0, n0, M, N, kbeg, kend, g.vec != 0, As,
                              Bs, acc);
  if (g.ksplit > 1) {
    // whole padded tile into this chunk's slot; rows and columns past M, N
    // hold zeros (out-of-range operands load as zero)
    const int64_t ldp = static_cast<int64_t>(g.tiles_m) * S::BM;
    const int64_t np = static_cast<int64_t>(g.tiles_n) * S::BN;
    double* P = g.part + kz * ldp * np;
#pragma unroll
    for (int i = 0; i < S::IB; ++i)
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        store4(P, ldp, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), ldp, np, true, acc[i][j]);
    return;
  }
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < S::IB; ++i) {
    const int64_t row0 = m0 + acc_row0<S>(i);
    d4 old[S::JB];
#pragma unroll
    for (int j = 0; j < S::JB; ++j)
      old[j] = need ? load4(g.C, g.ldc, row0, n0 + acc_col<S>(j), M, N, vc)
                    : (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t col = n0 + acc_col<S>(j);
      d4 v;
      if (OP == kBatchNN) v = g.alpha * acc[i][j] + g.beta * old[j];
      else v = acc[i][j];
      store4(g.C, g.ldc, row0, col, M, N, vc, v);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < M && col < N) sq += v[r] * v[r];
    }
  }
  if (OP != kBatchNN && g.sq != nullptr) {
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) g.sq[t] = tot;
  }
}

// Units of a launch whose count is known only on the device (the
// device-planned batch loop keeps one grid while the work shrinks):
// workgroup g takes unit g first, then further units gridDim.x + (launch
// counter)++ one at a time, so the long units do not pile up on a few
// workgroups, and a workgroup with nothing to do (the tail of the batch)
// exits without touching the counter.  Thread 0 takes the next unit when it
// starts the current one, so the atomic's latency hides behind the unit's
// work; the workgroup reads it from LDS afterwards, made wave-uniform
// (readfirstlane) so that the descriptor and the addresses derived from it
// stay in scalar registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(
      static_cast<int>(static_cast<uint64_t>(v) & 0xffffffffu)));
  const uint32_t hi = static_cast<uint32_t>(
      __builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint64_t>(v) >> 32)));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <class Body>
__device__ __forceinline__ void walk_units(unsigned long long* next, int64_t n, int64_t* slot,
                                           Body&& body) {
  int64_t blk = blockIdx.x;
  while (blk < n) {
    unsigned long long nx = 0;
    if (threadIdx.x == 0) nx = atomicAdd(next, 1ull);
    body(blk);
    if (threadIdx.x == 0) *slot = static_cast<int64_t>(gridDim.x) + static_cast<int64_t>(nx);
    __syncthreads();
    blk = wave_uniform(*slot);
    __syncthreads();
  }
}

// Unit of workgroup L in a one-unit-per-workgroup launch of n units, or -1.
// Workgroups go to the eight XCDs round-robin (L % 8), each with its own
// L2; XCD x takes the contiguous units [x per, (x + 1) per), per =
// ceil(n / 8), in order, so the operands that a problem's units share (Q_i
// and B_i of the downdate, Q_i of B_i = Q_i^T R, the sketch of R Omega) are
// fetched into one L2 rather than into all eight.  Needs a grid that is a
// multiple of 8 and at least n.
__device__ __forceinline__ int64_t xcd_unit(int64_t L, int64_t n) {
  const int64_t per = (n + 7) >> 3;
  const int64_t u = (L & 7) * per + (L >> 3);
  return (L >> 3) < per && u < n ? u : -1;
}

// WALK false: one unit per workgroup; the grid is an upper bound on the
// launch's units (planned on the host from the widest step any problem still
// active could take), and the workgroups past the device count exit at once.
// WALK true: a grid smaller than that bound walks the units (walk_units).
template <class S, int OP, bool WALK>
__global__ __launch_bounds__(S::NT, S::OCC) void gemm_batched_kernel(
    const BatchGemm* __restrict__ desc, int count, const int64_t* __restrict__ total,
    unsigned long long* __restrict__ next) {
  __shared__ __attribute__((aligned(16))) double lds[BatchLds<S>::kSize];
  __shared__ double red[S::NT / 64];
  double* As = lds;
  double* Bs = lds + 2 * S::A_LDS;
  if constexpr (!WALK) {
    const int64_t blk = xcd_unit(blockIdx.x, *total);
    if (blk >= 0) batched_tile<S, OP>(desc, count, blk, As, Bs, red);
  } else {
    __shared__ int64_t slot;
    walk_units(next, *total, &slot,
               [&](int64_t blk) { batched_tile<S, OP>(desc, count, blk, As, Bs, red); });
  }
}

// C from the depth chunks of the problems with ksplit > 1, in chunk order;
// kBatchRed elements of C per unit
template <int OP>
__device__ __forceinline__ void batched_reduce_unit(const BatchGemm* __restrict__ desc, int count,
                                                    int64_t blk, double* red) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {  // last problem with rblock0 <= blk
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].rblock0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  const BatchGemm g = desc[lo];
  const int64_t rb = blk - g.rblock0;
  const int64_t M = g.M, total = M * g.N;
  const int64_t ldp = static_cast<int64_t>(g.tiles_m) * g.bm;
  const int64_t slot = ldp * (static_cast<int64_t>(g.tiles_n) * g.bn);
  double sq = 0.0;
#pragma unroll
  for (int q = 0; q < kBatchRed / 256; ++q) {
    const int64_t e = rb * kBatchRed + q * 256 + threadIdx.x;
    if (e < total) {
      const int64_t i = e % M, j = e / M;
      const double* p = g.part + i + j * ldp;
      double v = 0.0;
      for (int z = 0; z < g.ksplit; ++z) v += p[z * slot];
      double* c = g.C + i + j * g.ldc;
      if (OP == kBatchNN) v = g.alpha * v + (g.beta != 0.0 ? g.beta * *c : 0.0);
      *c = v;
      sq += v * v;
    }
  }
  if (g.sq != nullptr) {
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) g.sq[rb] = tot;
  }
}

template <int OP, bool WALK>
__global__ __launch_bounds__(256) void gemm_batched_reduce_kernel(
    const BatchGemm* __restrict__ desc, int count, const int64_t* __restrict__ total,
    unsigned long long* __restrict__ next) {
  __shared__ double red[4];
  if constexpr (!WALK) {
    const int64_t blk = blockIdx.x;
    if (blk < *total) batched_reduce_unit<OP>(desc, count, blk, red);
  } else {
    __shared__ int64_t slot;
    walk_units(next, *total, &slot,
               [&](int64_t blk) { batched_reduce_unit<OP>(desc, count, blk, red); });
  }
}

}  // namespace

namespace {
// Grids up to this many workgroups run one unit per workgroup; larger
// bounds are walked by kWalkGrid workgroups.
// QB_BATCHED_WALK (set) walks every launch, so the fallback runs on batches
// small enough for a test.
constexpr int64_t kWalkGrid = 2048;
int64_t exact_grid_max() {
  return getenv("QB_BATCHED_WALK") != nullptr ? 0 : (int64_t(1) << 22);
}

template <class S, bool WALK>
void launch_batched_as(int op, const BatchGemm* desc, int count, dim3 grid, const int64_t* total,
                       unsigned long long* next, hipStream_t s) {
  if (op == kBatchNN)
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchNN, WALK>), grid, dim3(S::NT), 0, s, desc,
                       count, total, next);
  else if (op == kBatchTN)
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchTN, WALK>), grid, dim3(S::NT), 0, s, desc,
                       count, total, next);
  else
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchDD, WALK>), grid, dim3(S::NT), 0, s, desc,
                       count, total, next);
}

template <class S>
void launch_batched(int op, const BatchGemm* desc, int count, int64_t bound, const int64_t* total,
                    unsigned long long* next, hipStream_t s) {
  if (bound <= exact_grid_max())  // a multiple of 8 for xcd_unit
    launch_batched_as<S, false>(op, desc, count, dim3(static_cast<unsigned>((bound + 7) & ~int64_t(7))),
                                total, next, s);
  else
    launch_batched_as<S, true>(op, desc, count, dim3(static_cast<unsigned>(kWalkGrid)), total,
                               next, s);
}
}  // namespace

static_assert(BatchG16::BM == 16 && BatchG16::BN == 16 && BatchG32::BM == 32 &&
                  BatchG32::BN == 32 && BatchN32::BM == 64 && BatchN32::BN == 32 &&
                  BatchM32::BM == 32 && BatchM32::BN == 64 && Small::BM == kBatchTile &&
                  Small::BN == kBatchTile,
              "batch_tile_dims_hd follows the tile shapes");

void batch_tile_dims(int cls, int* bm, int* bn) {
  switch (cls) {
    case kTileG16: *bm = BatchG16::BM; *bn = BatchG16::BN; return;
    case kTileG32: *bm = BatchG32::BM; *bn = BatchG32::BN; return;
    case kTileN32: *bm = BatchN32::BM; *bn = BatchN32::BN; return;
    case kTileM32: *bm = BatchM32::BM; *bn = BatchM32::BN; return;
    default: *bm = Small::BM; *bn = Small::BN; return;
  }
}

int gemm_batched(int op, int cls, const BatchGemm* desc, int count, int64_t total_tiles,
                 int prof_id, double flops, double bytes, hipStream_t s,
                 const int64_t* dev_total, unsigned long long* dev_next) {
  if (count <= 0 || total_tiles <= 0) return kOk;
  if (op == kBatchDD && cls == kTileG16) return kEInval;
  if (dev_total == nullptr || dev_next == nullptr) return kEInval;
  ProfScope ps(prof_id, flops, bytes, s);
  switch (cls) {
    case kTileG16: launch_batched<BatchG16>(op, desc, count, total_tiles, dev_total, dev_next, s); break;
    case kTileG32: launch_batched<BatchG32>(op, desc, count, total_tiles, dev_total, dev_next, s); break;
    case kTileN32: launch_batched<BatchN32>(op, desc, count, total_tiles, dev_total, dev_next, s); break;
    case kTileM32: launch_batched<BatchM32>(op, desc, count, total_tiles, dev_total, dev_next, s); break;
    default: launch_batched<Small>(op, desc, count, total_tiles, dev_total, dev_next, s); break;
  }
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int gemm_batched_reduce(int op, const BatchGemm* desc, int count, int64_t total_rblocks,
                        int prof_id, hipStream_t s, const int64_t* dev_total,
                        unsigned long long* dev_next) {
  if (count <= 0 || total_rblocks <= 0) return kOk;
  if (op == kBatchDD || dev_total == nullptr || dev_next == nullptr) return kEInval;
  const bool walk = total_rblocks > exact_grid_max();
  const dim3 grid(static_cast<unsigned>(walk ? kWalkGrid : total_rblocks));
  ProfScope ps(prof_id, 0.0, 0.0, s);
  if (op == kBatchNN) {
    if (walk)
      hipLaunchKernelGGL((gemm_batched_reduce_kernel<kBatchNN, true>), grid, dim3(256), 0, s, desc,
                         count, dev_total, dev_next);
    else
      hipLaunchKernelGGL((gemm_batched_reduce_kernel<kBatchNN, false>), grid, dim3(256), 0, s,
                         desc, count, dev_total, dev_next);
  } else {
    if (walk)
      hipLaunchKernelGGL((gemm_batched_reduce_kernel<kBatchTN, true>), grid, dim3(256), 0, s, desc,
                         count, dev_total, dev_next);
    else
      hipLaunchKernelGGL((gemm_batched_reduce_kernel<kBatchTN, false>), grid, dim3(256), 0, s,
                         desc, count, dev_total, dev_next);
  }
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

}  // namespace qb
