// Batched FP64 MFMA products: every active problem's product of one step of
// the batched block loop in one launch.  Workgroup -> (problem, tile, depth
// chunk) by binary search over the problems' first workgroup indices; the
// tile loop and epilogues are those of the single-matrix kernels
// (gemm_tiles.hpp).  Problems whose product is split over depth chunks
// leave their partial tiles to gemm_batched_reduce, which sums them in chunk
// order, so results are bitwise reproducible.
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
  const bool vc = vec_ok_dev(g.C, g.ldc);
  const bool need = g.ksplit == 1 && ((OP == kBatchDD) || (OP == kBatchNN && g.beta != 0.0));
  // a downdate reads its old C tile before the MMA loop, so the read latency
  // overlaps the operand loads (69 against 74 ms per 512-problem batch, at
  // three workgroups per CU for the extra registers instead of four; half
  // the tile read ahead at four workgroups per CU: 76 ms); the other
  // products read it in the epilogue and keep four
  constexpr bool kAhead = OP == kBatchDD;
  d4 ahead[kAhead ? S::IB : 1][S::JB];
  if constexpr (kAhead) {
#pragma unroll
    for (int i = 0; i < S::IB; ++i)
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        ahead[i][j] = need ? load4(g.C, g.ldc, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, vc)
                           : (d4){0.0, 0.0, 0.0, 0.0};
  }
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
    for (int j = 0; j < S::JB; ++j) {
      if constexpr (kAhead) old[j] = ahead[i][j];
      else old[j] = need ? load4(g.C, g.ldc, row0, n0 + acc_col<S>(j), M, N, vc)
                         : (d4){0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t col = n0 + acc_col<S>(j);
      d4 v;
      if (OP == kBatchNN) v = g.alpha * acc[i][j] + g.beta * old[j];
      else if (OP == kBatchTN) v = acc[i][j];
      else v = old[j] - acc[i][j];
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

// total: null for one workgroup per (problem, tile, chunk) (grid = the
// total); else the device count of such units, which a grid of any size
// walks in strides of the grid (the device-planned batch loop, whose
// launches keep one grid while the work shrinks)
// Units of a launch whose count is known only on the device: workgroup g
// takes unit g first, then further units gridDim.x + (launch counter)++ one
// at a time, so the long units do not pile up on a few workgroups, and a
// workgroup with nothing to do (the tail of the batch) exits without
// touching the counter.  Thread 0 takes the next unit when it starts the
// current one, so the atomic's latency hides behind the unit's work; the
// workgroup reads it from LDS afterwards.
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
    blk = *slot;
    __syncthreads();
  }
}

template <class S, int OP>
__global__ __launch_bounds__(S::NT, S::OCC) void gemm_batched_kernel(
    const BatchGemm* __restrict__ desc, int count, const int64_t* __restrict__ total,
    unsigned long long* __restrict__ next) {
  __shared__ __attribute__((aligned(16))) double As[2 * S::A_LDS];
  __shared__ __attribute__((aligned(16))) double Bs[2 * S::B_LDS];
  __shared__ double red[S::NT / 64];
  __shared__ int64_t slot;
  if (total == nullptr) {
    batched_tile<S, OP>(desc, count, blockIdx.x, As, Bs, red);
    return;
  }
  // units of very different depth: taken one at a time from a counter, so
  // the long ones do not pile up on a few workgroups
  walk_units(next, *total, &slot,
             [&](int64_t blk) { batched_tile<S, OP>(desc, count, blk, As, Bs, red); });
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

template <int OP>
__global__ __launch_bounds__(256) void gemm_batched_reduce_kernel(
    const BatchGemm* __restrict__ desc, int count, const int64_t* __restrict__ total,
    unsigned long long* __restrict__ next) {
  __shared__ double red[4];
  __shared__ int64_t slot;
  if (total == nullptr) {
    batched_reduce_unit<OP>(desc, count, blockIdx.x, red);
    return;
  }
  walk_units(next, *total, &slot,
             [&](int64_t blk) { batched_reduce_unit<OP>(desc, count, blk, red); });
}

}  // namespace

namespace {
template <class S>
void launch_batched(int op, const BatchGemm* desc, int count, int64_t grid_size,
                    const int64_t* total, unsigned long long* next, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(grid_size));
  if (op == kBatchNN)
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchNN>), grid, dim3(S::NT), 0, s, desc, count,
                       total, next);
  else if (op == kBatchTN)
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchTN>), grid, dim3(S::NT), 0, s, desc, count,
                       total, next);
  else
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchDD>), grid, dim3(S::NT), 0, s, desc, count,
                       total, next);
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
  if (total_tiles > INT32_MAX) return kEInval;  // one-dimensional grid
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
  if (total_rblocks > INT32_MAX) return kEInval;
  if (op == kBatchDD) return kEInval;
  const dim3 grid(static_cast<unsigned>(total_rblocks));
  ProfScope ps(prof_id, 0.0, 0.0, s);
  if (op == kBatchNN)
    hipLaunchKernelGGL(gemm_batched_reduce_kernel<kBatchNN>, grid, dim3(256), 0, s, desc, count,
                       dev_total, dev_next);
  else
    hipLaunchKernelGGL(gemm_batched_reduce_kernel<kBatchTN>, grid, dim3(256), 0, s, desc, count,
                       dev_total, dev_next);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

}  // namespace qb
