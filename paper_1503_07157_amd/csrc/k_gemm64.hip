// FP64 MFMA GEMM kernels of the blocked QB hot path (gfx950).
//
// Every product of Figure 4 / Figure 6 has one long side and one side of at
// most b (<= 256) columns:
//   gemm_nn   Y = X W            A Omega_i, A Z, Qbar C, Y T^{-1}   (K = long or b)
//   gemm_tn   C = Q^T X          Q_i^T A, Q_i^T Qbar, Y^T Y         (K = m, long)
//   downdate  R = R - Q_i B_i    with the fused residual sum of squares
// A workgroup of 256 threads (4 waves, 2 x 2) owns a BM x BN output tile
// (128 x 128 for the bulk products, 64 x 64 for small outputs); each wave
// owns a (BM/2) x (BN/2) sub-tile as 16 x 16 blocks of
// v_mfma_f64_16x16x4_f64.  Operand tiles of depth 16 pass through two LDS
// stages with register prefetch of the slice after; one LDS-only barrier
// per slice.  Long reductions are split over workgroups (split-K) into
// partial buffers that a second kernel sums in a fixed order, so results
// are bitwise reproducible run to run.
//
// Tile shapes, operand staging and the MFMA depth loop: gemm_tiles.hpp.
#include <cstdlib>

#include "gemm_tiles.hpp"

namespace qb {
namespace {

// ---------------------------------------------------------------------------
// Y = alpha X W + beta Y   (X: M x K m-contiguous, W: K x N, k-contiguous)
// grid: (M tiles, N tiles, split); split > 1 writes part[z] (M x N, ld ldp)
template <class S>
__global__ __launch_bounds__(S::NT, S::OCC) void gemm_nn_kernel(const double* __restrict__ X, int64_t ldx,
                                                        const double* __restrict__ W, int64_t ldw,
                                                        double* __restrict__ Y, int64_t ldy,
                                                        int64_t M, int64_t N, int64_t K,
                                                        int64_t kchunk, double alpha, double beta,
                                                        double* __restrict__ part, int64_t ldp,
                                                        int vec_y, int vec_ab) {
  __shared__ __attribute__((aligned(16))) double As[2 * S::A_LDS];
  __shared__ __attribute__((aligned(16))) double Bs[2 * S::B_LDS];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * S::BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * S::BN;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  d4 acc[S::IB][S::JB];
  mma_loop<S, false>(X, ldx, W, ldw, m0, n0, M, N, kbeg, kend, vec_ab != 0, As, Bs, acc);
  if (part != nullptr) {
    double* P = part + static_cast<int64_t>(blockIdx.z) * ldp * N;
#pragma unroll
    for (int i = 0; i < S::IB; ++i)
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        store4(P, ldp, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, true, acc[i][j]);
  } else {
#pragma unroll
    for (int i = 0; i < S::IB; ++i) {
      d4 old[S::JB];
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        old[j] = (beta != 0.0)
                     ? load4(Y, ldy, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, vec_y)
                     : (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        store4(Y, ldy, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, vec_y,
               alpha * acc[i][j] + beta * old[j]);
    }
  }
}

// C = Q^T X  (Q: K x P so A = Q^T is k-contiguous; X: K x N)
// grid: (N tiles, P tiles, split)
template <class S>
__global__ __launch_bounds__(S::NT, S::OCC) void gemm_tn_kernel(const double* __restrict__ Qm, int64_t ldq,
                                                        const double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ C, int64_t ldc,
                                                        int64_t P, int64_t N, int64_t K,
                                                        int64_t kchunk, int transpose_out,
                                                        double* __restrict__ part, int64_t ldp,
                                                        double* __restrict__ sq_part, int vec_c,
                                                        int vec_ab) {
  __shared__ __attribute__((aligned(16))) double As[2 * S::A_LDS];
  __shared__ __attribute__((aligned(16))) double Bs[2 * S::B_LDS];
  __shared__ double red[S::NT / 64];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * S::BN;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * S::BM;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  d4 acc[S::IB][S::JB];
  mma_loop<S, true>(Qm, ldq, X, ldx, m0, n0, P, N, kbeg, kend, vec_ab != 0, As, Bs, acc);
  if (part != nullptr) {
    double* Pp = part + static_cast<int64_t>(blockIdx.z) * ldp * N;
#pragma unroll
    for (int i = 0; i < S::IB; ++i)
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        store4(Pp, ldp, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), P, N, true, acc[i][j]);
    return;
  }
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t row0 = m0 + acc_row0<S>(i), col = n0 + acc_col<S>(j);
      if (transpose_out) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row0 + r < P && col < N) C[col + (row0 + r) * ldc] = acc[i][j][r];
      } else {
        store4(C, ldc, row0, col, P, N, vec_c, acc[i][j]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < P && col < N) sq += acc[i][j][r] * acc[i][j][r];
    }
  if (sq_part != nullptr) {
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) sq_part[blockIdx.x + static_cast<int64_t>(blockIdx.y) * gridDim.x] = tot;
  }
}

// ---------------------------------------------------------------------------
// Stream-K form of the split products.  The depth of every output tile is
// cut into slices of BK; the slices of all tiles, tile after tile (tiles in
// column-major order over the output), are dealt to `groups` workgroups in
// runs of equal length (to within one slice).  Every workgroup then does
// the same work, where a whole number of splits per tile leaves part of
// the chip idle (40 tiles of 256 x 128 x 6 splits = 240 workgroups for
// 256 CUs).  A run crosses at most one tile boundary;
// each part of a run is stored as a partial tile in slice
// z = g - (first workgroup of that tile), and the reduce adds the tile's
// slices in order of z, so results are reproducible run to run.
struct StreamK {
  int64_t ut;       // depth slices per tile; 0 selects the plain split-K grid
  int64_t units;    // tiles * ut
  int64_t groups;   // workgroups
  int64_t tiles_m;  // tiles along the output rows
};

__host__ __device__ inline int64_t sk_start(const StreamK& k, int64_t g) {
  return g * k.units / k.groups;
}

// workgroup whose run holds slice u: the largest g with
// floor(g units / groups) <= u, i.e. ceil((u + 1) groups / units) - 1; in
// 32-bit arithmetic when the products fit
__host__ __device__ inline int64_t sk_owner(const StreamK& k, int64_t u) {
  if (k.units * k.groups <= int64_t(0xffffffff))
    return static_cast<int64_t>((static_cast<uint32_t>(u + 1) * static_cast<uint32_t>(k.groups) - 1u) /
                                static_cast<uint32_t>(k.units));
  return ((u + 1) * k.groups - 1) / k.units;
}

// partial slices that tile t receives
__host__ __device__ inline int64_t sk_pieces(const StreamK& k, int64_t t) {
  return sk_owner(k, (t + 1) * k.ut - 1) - sk_owner(k, t * k.ut) + 1;
}

// One part of a run: slices [u, u1) of tile t into partial slice z.
template <class S, bool TN>
__device__ __forceinline__ void sk_segment(const double* __restrict__ A, int64_t lda,
                                           const double* __restrict__ B, int64_t ldb, int64_t M,
                                           int64_t N, int64_t K, const StreamK& sk, int64_t t,
                                           int64_t u, int64_t u1, int64_t z,
                                           double* __restrict__ part, int64_t ldp, bool vec,
                                           double* As, double* Bs) {
  const int64_t tb = t * sk.ut;
  const int64_t m0 = (t % sk.tiles_m) * S::BM, n0 = (t / sk.tiles_m) * S::BN;
  const int64_t kbeg = (u - tb) * BK;
  const int64_t kend = ((u1 - tb) * BK < K) ? (u1 - tb) * BK : K;
  d4 acc[S::IB][S::JB];
  mma_loop<S, TN>(A, lda, B, ldb, m0, n0, M, N, kbeg, kend, vec, As, Bs, acc);
  double* Pz = part + z * ldp * N;
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j)
      store4(Pz, ldp, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, true, acc[i][j]);
}

// partial tiles of C = op(A) B over the run of workgroup blockIdx.x (at
// most two parts, as runs are shorter than a tile's depth); TN selects the
// k-contiguous A of gemm_tn (A = Q^T), else A is m-contiguous
template <class S, bool TN>
__global__ __launch_bounds__(S::NT, S::OCC) void gemm_sk_kernel(
    const double* __restrict__ A, int64_t lda, const double* __restrict__ B, int64_t ldb,
    int64_t M, int64_t N, int64_t K, StreamK sk, double* __restrict__ part, int64_t ldp,
    int vec_ab) {
  __shared__ __attribute__((aligned(16))) double As[2 * S::A_LDS];
  __shared__ __attribute__((aligned(16))) double Bs[2 * S::B_LDS];
  const int64_t g = blockIdx.x;
  const int64_t u0 = sk_start(sk, g), uend = sk_start(sk, g + 1);
  const int64_t t0 = u0 / sk.ut;
  const int64_t split = (t0 + 1) * sk.ut;  // first slice of the next tile
  if (split < uend) {
    // second part first: it starts a tile, so this workgroup owns slice 0
    sk_segment<S, TN>(A, lda, B, ldb, M, N, K, sk, t0 + 1, split, uend, 0, part, ldp,
                      vec_ab != 0, As, Bs);
    __syncthreads();  // the first part refills the LDS stages
  }
  sk_segment<S, TN>(A, lda, B, ldb, M, N, K, sk, t0, u0, split < uend ? split : uend,
                    g - sk_owner(sk, t0 * sk.ut), part, ldp, vec_ab != 0, As, Bs);
}

// out(M x N) = alpha * sum_s part[s] + beta * out; part[s] has ld ldp;
// transposed store puts element (i, j) at out[j + i*ldo].  Optional
// per-block sums of squares of the result.  In stream-K form (sk.ut > 0)
// the element's tile (bm x bn tiles) has its own number of slices.
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int split,
                                                     int64_t ldp, double* __restrict__ out,
                                                     int64_t ldo, int64_t M, int64_t N,
                                                     double alpha, double beta, int transpose_out,
                                                     double* __restrict__ sq_part, StreamK sk,
                                                     int bm, int bn) {
  __shared__ double red[4];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = M * N;
  double sq = 0.0;
  if (idx < total) {
    // (row, column) of the element; 32-bit division when the output fits
    int64_t i, j;
    if (total <= int64_t(0xffffffff)) {
      const uint32_t u = static_cast<uint32_t>(idx), mm = static_cast<uint32_t>(M);
      i = u % mm;
      j = u / mm;
    } else {
      i = idx % M;
      j = idx / M;
    }
    const int64_t pidx = i + j * ldp, pstride = ldp * N;
    // tile of the element: row and column below 2^31, so 32-bit division
    const int64_t nzs =
        sk.ut > 0 ? sk_pieces(sk, int64_t(static_cast<uint32_t>(j) / static_cast<uint32_t>(bn)) *
                                          sk.tiles_m +
                                      static_cast<uint32_t>(i) / static_cast<uint32_t>(bm))
                  : split;
    double s = 0.0;
    for (int64_t z = 0; z < nzs; ++z) s += part[z * pstride + pidx];
    const int64_t o = transpose_out ? (j + i * ldo) : (i + j * ldo);
    double v = alpha * s;
    if (beta != 0.0) v += beta * out[o];
    out[o] = v;
    sq = v * v;
  }
  if (sq_part != nullptr) {
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) sq_part[blockIdx.x] = tot;
  }
}

// The same sum for small outputs with many partials (the w x w Gram
// matrices): a workgroup covers 256 / G outputs with G threads each; thread
// g adds partials g, g + G, g + 2G, ... in increasing order and the G
// partial sums are added in the order g = 0 .. G-1.  A fixed order, so the
// result is the same on every run.
template <int G>
__global__ __launch_bounds__(256) void reduce_wide_kernel(const double* __restrict__ part,
                                                          int split, int64_t ldp,
                                                          double* __restrict__ out, int64_t ldo,
                                                          int64_t M, int64_t N, double alpha,
                                                          double beta, int transpose_out) {
  constexpr int OPB = 256 / G;
  __shared__ double buf[G][OPB];
  const int o = threadIdx.x % OPB, g = threadIdx.x / OPB;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * OPB + o;
  const int64_t total = M * N;
  const int64_t i = idx % M, j = idx / M;
  double s = 0.0;
  if (idx < total) {
    const int64_t pstride = ldp * N;
    const double* pp = part + i + j * ldp;
#pragma unroll 4
    for (int z = g; z < split; z += G) s += pp[z * pstride];
  }
  buf[g][o] = s;
  __syncthreads();
  if (g == 0 && idx < total) {
    double v = buf[0][o];
#pragma unroll
    for (int q = 1; q < G; ++q) v += buf[q][o];
    v *= alpha;
    const int64_t oi = transpose_out ? (j + i * ldo) : (i + j * ldo);
    if (beta != 0.0) v += beta * out[oi];
    out[oi] = v;
  }
}

constexpr int kWideG = 8;  // threads per output in reduce_wide_kernel

// launch the split-K sum; the wide form serves small outputs with many
// partials when no per-block sums of squares are asked for
void launch_reduce(const double* part, int nz, int64_t ldp, double* out, int64_t ldo, int64_t M,
                   int64_t N, double alpha, double beta, bool tr, double* sq_part, unsigned* nb,
                   hipStream_t s, const StreamK& sk = StreamK{0, 0, 0, 0}, int bm = 1,
                   int bn = 1) {
  const int64_t total = M * N;
  if (sk.ut == 0 && sq_part == nullptr && nz >= 2 * kWideG && total <= (int64_t(1) << 18)) {
    constexpr int OPB = 256 / kWideG;
    *nb = static_cast<unsigned>(cdiv(total, OPB));
    hipLaunchKernelGGL(reduce_wide_kernel<kWideG>, dim3(*nb), dim3(256), 0, s, part, nz, ldp, out,
                       ldo, M, N, alpha, beta, tr ? 1 : 0);
    return;
  }
  *nb = static_cast<unsigned>(cdiv(total, 256));
  hipLaunchKernelGGL(reduce_kernel, dim3(*nb), dim3(256), 0, s, part, nz, ldp, out, ldo, M, N,
                     alpha, beta, tr ? 1 : 0, sq_part, sk, bm, bn);
}

// Tile order of the downdate: the eight XCDs (workgroup L runs on XCD
// L % 8, each with its own 4 MB L2) take contiguous ranges of one sequence,
// which runs over groups of G row tiles (kDdRows rows of R), each group
// swept across all column tiles.  An XCD then holds its group's Q row
// blocks (2 MB at depth 256) in L2 while the B column blocks stream past.
// With the plain (row tile, column tile) grid every XCD walked every eighth
// row tile of each column, touched 5 MB of Q row blocks per column at
// b = 256 and fetched them again for the next: 3.0x the algorithmic bytes
// per launch at 20000 x 16000 (FETCH_SIZE/WRITE_SIZE), 1.65x in this order.
constexpr int64_t kDdRows = 1024;
__device__ __forceinline__ bool dd_tile(int64_t L, int64_t tm, int64_t tn, int64_t G, int64_t* row,
                                        int64_t* col) {
  const int64_t total = tm * tn;
  const int64_t per = (total + 7) >> 3;
  const int64_t j = L >> 3;
  const int64_t u = (L & 7) * per + j;
  if (j >= per || u >= total) return false;
  const int64_t span = G * tn;
  const int64_t grp = u / span, w = u - grp * span;
  const int64_t rows = tm - grp * G < G ? tm - grp * G : G;
  *col = w / rows;
  *row = grp * G + (w - *col * rows);
  return true;
}

// R -= Q B; per-workgroup sum of squares of the updated tile, at index
// row tile + column tile * (row tiles).  grid: 8 ceil(tiles / 8), one
// dimension (dd_tile).  AHEAD: the R tile is read before the depth loop
// (its latency overlaps the MFMA work; registers for the whole tile, so
// 64 x 64 tiles only); else it is read in the epilogue.
template <class S, bool AHEAD>
__global__ __launch_bounds__(S::NT, S::OCC) void downdate_kernel(double* __restrict__ R, int64_t ldr,
                                                         const double* __restrict__ Qm,
                                                         int64_t ldq,
                                                         const double* __restrict__ B,
                                                         int64_t ldb, int64_t M, int64_t N,
                                                         int64_t K,
                                                         double* __restrict__ sq_part,
                                                         int vec_r, int vec_ab) {
  __shared__ __attribute__((aligned(16))) double As[2 * S::A_LDS];
  __shared__ __attribute__((aligned(16))) double Bs[2 * S::B_LDS];
  __shared__ double red[S::NT / 64];
  const int64_t tm = (M + S::BM - 1) / S::BM, tn = (N + S::BN - 1) / S::BN;
  int64_t tr = 0, tc = 0;
  if (!dd_tile(blockIdx.x, tm, tn, kDdRows / S::BM, &tr, &tc)) return;
  const int64_t m0 = tr * S::BM;
  const int64_t n0 = tc * S::BN;
  d4 rv[AHEAD ? S::IB : 1][S::JB];
  if constexpr (AHEAD) {
#pragma unroll
    for (int i = 0; i < S::IB; ++i)
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        rv[i][j] = load4(R, ldr, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, vec_r);
  }
  d4 acc[S::IB][S::JB];
  mma_loop<S, false>(Qm, ldq, B, ldb, m0, n0, M, N, 0, K, vec_ab != 0, As, Bs, acc);
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < S::IB; ++i) {
    const int64_t row0 = m0 + acc_row0<S>(i);
    if constexpr (!AHEAD) {
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        rv[0][j] = load4(R, ldr, row0, n0 + acc_col<S>(j), M, N, vec_r);
    }
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t col = n0 + acc_col<S>(j);
      const d4 v = rv[AHEAD ? i : 0][j] - acc[i][j];
      store4(R, ldr, row0, col, M, N, vec_r, v);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < M && col < N) sq += v[r] * v[r];
    }
  }
  const double tot = block_sum(sq, red);
  if (threadIdx.x == 0) sq_part[tr + tc * tm] = tot;
}

int64_t part_ld(int64_t M) { return (M + 1) & ~int64_t(1); }

int64_t kchunk_for(int64_t K, int split) {
  const int64_t c = cdiv(K, split);
  return cdiv(c, BK) * BK;
}

int vec_ok(const double* p, int64_t ld) {
  return ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && (ld & 1) == 0) ? 1 : 0;
}

// tile loads use 32-bit element offsets: 128 rows/columns times ld must fit
bool ld_fits(int64_t ld) { return ld >= 0 && ld < (int64_t(1) << 24); }

// Tall tiles for gemm_nn when there are enough of them for one workgroup
// per CU: measured 465 us against 579 us for the 10000 x 10000 x 128 split-K
// product, the A slices being read as whole 2 KB DRAM pages
bool use_tall(int64_t M, int64_t N, int nz) {
  return cdiv(M, Tall::BM) * cdiv(N, Tall::BN) * nz >= int64_t(7) * kNumCU / 8;
}

template <class S>
void launch_nn(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y,
               int64_t ldy, int64_t M, int64_t N, int64_t K, int64_t kc, int nz, double alpha,
               double beta, double* part, int64_t ldp, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(cdiv(M, S::BM)), static_cast<unsigned>(cdiv(N, S::BN)),
                  static_cast<unsigned>(nz));
  hipLaunchKernelGGL(gemm_nn_kernel<S>, grid, dim3(S::NT), 0, s, X, ldx, W, ldw, Y, ldy, M, N, K,
                     kc, alpha, beta, part, ldp, vec_ok(Y, ldy), vec_ok(X, ldx) & vec_ok(W, ldw));
}

template <class S>
dim3 launch_tn(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C,
               int64_t ldc, int64_t P, int64_t N, int64_t K, int64_t kc, int nz, bool tr,
               double* part, int64_t ldp, double* sq_part, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(cdiv(N, S::BN)), static_cast<unsigned>(cdiv(P, S::BM)),
                  static_cast<unsigned>(nz));
  hipLaunchKernelGGL(gemm_tn_kernel<S>, grid, dim3(S::NT), 0, s, Qm, ldq, X, ldx, C, ldc, P, N, K,
                     kc, tr ? 1 : 0, part, ldp, sq_part, vec_ok(C, ldc),
                     vec_ok(Qm, ldq) & vec_ok(X, ldx));
  return grid;
}

// Stream-K plan for an M x N x K product split `split` ways: one workgroup
// per resident place (at most tiles * (split + 1) - 1 of them, so that no
// tile receives more than split + 2 partial slices, the size of the
// partial buffer); ut = 0 (the plain grid) when the runs would be shorter
// than two slices or the tiles already fill the places.
template <class S>
StreamK plan_sk(int64_t M, int64_t N, int64_t K, int split) {
  const StreamK none{0, 0, 0, 0};
  if (M >= (int64_t(1) << 31) || N >= (int64_t(1) << 31)) return none;  // 32-bit tile index
  const int64_t tm = cdiv(M, S::BM), tiles = tm * cdiv(N, S::BN);
  const int64_t ut = cdiv(K, BK);
  int64_t g = int64_t(kNumCU) * S::OCC;
  if (g > tiles * (split + 1) - 1) g = tiles * (split + 1) - 1;
  if (split < 2 || g <= tiles || tiles * ut < 2 * g) return none;
  const StreamK sk{ut, tiles * ut, g, tm};
  for (int64_t t = 0; t < tiles; ++t)
    if (sk_pieces(sk, t) > split + 2) return none;
  return sk;
}

template <class S, bool TN>
void launch_sk(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
               int64_t K, const StreamK& sk, double* part, int64_t ldp, hipStream_t s) {
  hipLaunchKernelGGL((gemm_sk_kernel<S, TN>), dim3(static_cast<unsigned>(sk.groups)),
                     dim3(S::NT), 0, s, A, lda, B, ldb, M, N, K, sk, part, ldp,
                     vec_ok(A, lda) & vec_ok(B, ldb));
}

}  // namespace

int choose_split(int64_t M, int64_t N, int64_t K, int slots_per_cu, bool tall_nn) {
  // Workgroups resident at once: 256 CUs x slots_per_cu.  A split that
  // leaves a partial second round costs as much as a full one, so take the
  // largest split that still fits in one round of 128 x 128 tiles
  // (QB_SPLIT_TARGET overrides the number of resident workgroups).
  static const int64_t target = [] {
    const char* e = getenv("QB_SPLIT_TARGET");
    const long v = e ? atol(e) : 0;
    return v > 0 ? static_cast<int64_t>(v) : int64_t(0);
  }();
  const int64_t slots = target > 0 ? target : int64_t(kNumCU) * slots_per_cu;
  const int64_t tiles = cdiv(M, kTileM) * cdiv(N, kTileN);
  int64_t s = tiles > 0 ? slots / tiles : 1;
  const int64_t by_depth = K / kSplitMinDepth;
  if (s > by_depth) s = by_depth;
  const int64_t by_mem = kPartialCapDoubles / ((M * N > 0) ? M * N : 1);
  if (s > by_mem) s = by_mem;
  if (s > kMaxSplit) s = kMaxSplit;
  if (s < 1) s = 1;
  // A tall product with a narrow output (Y = R Omega_i, Qbar C at b = 256:
  // 314 tiles of 128 x 128) fills between one and two rounds of 128 x 128
  // tiles, so the rule above leaves it unsplit and 40 % of the places idle
  // (28 TF/s measured at 20000 x 16000 x 256).  A split of two lets gemm_nn
  // deal its depth out stream-K over one 256 x 128 workgroup per CU
  // (tall_nn: callers whose product runs on gemm_nn).
  if (tall_nn && s == 1 && M >= 8 * N && N <= kMaxPanel && by_depth >= 2 && by_mem >= 2 &&
      cdiv(M, 256) * cdiv(N, kTileN) * 2 >= int64_t(7) * kNumCU / 8)
    s = 2;
  return static_cast<int>(s);
}

// Split for the low-precision sampling kernels (128 x 128 tiles, no
// stream-K): the split, within the depth and partial-memory limits, whose
// workgroups fill their last round of slots best (ties to the smaller).
// 314 tiles on 512 slots (Y = R Omega at 20000 x 256): 1 and 2 fill 61 %,
// 3 fills 92 %.
int choose_split_fill(int64_t M, int64_t N, int64_t K, int slots_per_cu, int bm, int bn) {
  const int64_t slots = int64_t(kNumCU) * slots_per_cu;
  const int64_t tiles = cdiv(M, bm) * cdiv(N, bn);
  int64_t lim = K / kSplitMinDepth;
  const int64_t by_mem = kPartialCapDoubles / ((M * N > 0) ? M * N : 1);
  if (lim > by_mem) lim = by_mem;
  if (lim > 8) lim = 8;
  int best = 1;
  double best_fill = 0.0;
  for (int64_t s = 1; s <= (lim < 1 ? 1 : lim); ++s) {
    const int64_t wg = tiles * s, rounds = cdiv(wg, slots);
    const double fill = double(wg) / double(rounds * slots);
    if (fill > best_fill + 1e-9) {
      best_fill = fill;
      best = static_cast<int>(s);
    }
  }
  return best;
}

// split slices, and two more for the stream-K form
size_t partial_doubles(int64_t M, int64_t N, int split) {
  return split > 1 ? static_cast<size_t>(part_ld(M)) * N * (split + 2) : 0;
}

int gemm_nn(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y, int64_t ldy,
            int64_t M, int64_t N, int64_t K, double alpha, double beta, int split, double* part,
            hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  if (!ld_fits(ldx) || !ld_fits(ldw)) return kEInval;
  if (K <= 0) split = 1;
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? kchunk_for(K, split) : (K > 0 ? K : 0);
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  const int64_t ldp = part_ld(M);
  // unsplit products with too few 128 x 128 tiles to fill the chip twice
  // (the T^{-1} application, short projections) take 64 x 64 tiles: at
  // 20000 x 256 x 256 the 314 tiles of 128 x 128 left most of a second
  // round of 256 CUs idle (T^{-1} applications 21.8 -> 13.8 ms per 20000 x
  // 16000 factorisation in 64 x 64 tiles); tall products with enough
  // 256-row tiles for one workgroup per CU take Tall
  const bool small = nz == 1 && cdiv(M, Big::BM) * cdiv(N, Big::BN) < 2 * kNumCU;
  const bool tall = !small && use_tall(M, N, nz);
  // stream-K for the tall tiles only (measured: 89 -> 86 ms of sampling
  // products per 10000 x 10000 factorisation); the 128 x 128 forms spill
  // registers when they handle two parts of a run, and gemm_tn gained
  // nothing from it while its reduce read a quarter more partials
  const StreamK sk = (nz > 1 && tall) ? plan_sk<Tall>(M, N, K, split) : StreamK{0, 0, 0, 0};
  {
    ProfScope ps(small ? kKGemmNNSmall : tall ? kKGemmNNTall : kKGemmNN, 2.0 * M * N * K,
                 8.0 * (M * K + K * N + M * N * (beta != 0.0 ? 2 : 1)), s);
    double* pp = nz > 1 ? part : nullptr;
    if (small)
      launch_nn<Small>(X, ldx, W, ldw, Y, ldy, M, N, K, kc, nz, alpha, beta, pp, ldp, s);
    else if (sk.ut > 0)
      launch_sk<Tall, false>(X, ldx, W, ldw, M, N, K, sk, part, ldp, s);
    else if (tall)
      launch_nn<Tall>(X, ldx, W, ldw, Y, ldy, M, N, K, kc, nz, alpha, beta, pp, ldp, s);
    else
      launch_nn<Big>(X, ldx, W, ldw, Y, ldy, M, N, K, kc, nz, alpha, beta, pp, ldp, s);
  }
  QB_HIP_TRY(hipGetLastError());
  if (nz > 1) {
    const int64_t total = M * N;
    ProfScope ps(kKReduce, double(nz) * total, 8.0 * (nz + (beta != 0.0 ? 2 : 1)) * total, s);
    unsigned nb = 0;
    launch_reduce(part, nz, ldp, Y, ldy, M, N, alpha, beta, false, nullptr, &nb, s, sk, Tall::BM,
                  Tall::BN);
    QB_HIP_TRY(hipGetLastError());
  }
  return kOk;
}

int gemm_tn(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C, int64_t ldc,
            int64_t P, int64_t N, int64_t K, bool transpose_out, int split, double* part,
            double* sq_part, int* sq_count, hipStream_t s) {
  if (P <= 0 || N <= 0) { if (sq_count) *sq_count = 0; return kOk; }
  if (!ld_fits(ldq) || !ld_fits(ldx)) return kEInval;
  if (K <= 0) split = 1;
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? kchunk_for(K, split) : (K > 0 ? K : 0);
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  const int64_t ldp = part_ld(P);
  // small outputs (the w x w Gram matrices, Q_i^T Qbar early on) take
  // 64 x 64 tiles: four times the workgroups for the same split.  Products
  // that return per-tile sums of squares keep the 128 x 128 tiles the
  // partial-sum buffers are sized for.
  const bool small = P * N <= int64_t(256) * 256 && (sq_part == nullptr || nz > 1);
  // A panel of 129..256 columns (b = 256) takes 256-row tiles, so the long
  // operand X is read once per column tile instead of once per 128-row tile
  // row (counters at 20000 x 16000: 2.3x the algorithmic bytes with two
  // tile rows)
  const bool tall = !small && P > kTileM && P <= Tall::BM;
  dim3 grid;
  {
    ProfScope ps(small ? kKGemmTNSmall : kKGemmTN, 2.0 * P * N * K, 8.0 * (K * P + K * N + P * N), s);
    double* pp = nz > 1 ? part : nullptr;
    double* sqp = nz > 1 ? static_cast<double*>(nullptr) : sq_part;
    grid = small ? launch_tn<Small>(Qm, ldq, X, ldx, C, ldc, P, N, K, kc, nz, transpose_out, pp,
                                    ldp, sqp, s)
           : tall ? launch_tn<Tall>(Qm, ldq, X, ldx, C, ldc, P, N, K, kc, nz, transpose_out, pp,
                                    ldp, sqp, s)
                  : launch_tn<Big>(Qm, ldq, X, ldx, C, ldc, P, N, K, kc, nz, transpose_out, pp,
                                   ldp, sqp, s);
  }
  QB_HIP_TRY(hipGetLastError());
  if (nz > 1) {
    const int64_t total = P * N;
    unsigned nb = 0;
    ProfScope ps(kKReduce, double(nz) * total, 8.0 * (nz + 1) * total, s);
    launch_reduce(part, nz, ldp, C, ldc, P, N, 1.0, 0.0, transpose_out, sq_part, &nb, s);
    QB_HIP_TRY(hipGetLastError());
    if (sq_count) *sq_count = sq_part ? static_cast<int>(nb) : 0;
  } else {
    if (sq_count) *sq_count = sq_part ? static_cast<int>(grid.x * grid.y) : 0;
  }
  return kOk;
}

size_t downdate_partials(int64_t M, int64_t N) {  // the most tiles: 64 x 64
  return static_cast<size_t>(cdiv(M, Small::BM)) * static_cast<size_t>(cdiv(N, Small::BN));
}

int downdate(double* R, int64_t ldr, const double* Qm, int64_t ldq, const double* B, int64_t ldb,
             int64_t M, int64_t N, int64_t K, double* sq_part, int* sq_count, hipStream_t s) {
  if (M <= 0 || N <= 0) { if (sq_count) *sq_count = 0; return kOk; }
  if (!ld_fits(ldq) || !ld_fits(ldb)) return kEInval;
  // Shallow updates (K < 192): 64 x 64 tiles, each reading its R tile ahead
  // of the depth loop (measured per 10^4 x 10^4 factorisation at b = 128:
  // 51.7 -> 49.1 ms against 128 x 128 tiles with R read in the epilogue).
  // Deep ones with tiles for every CU: 128 x 128 tiles, two workgroups per
  // CU, R read in the epilogue (one workgroup's epilogue overlaps the other's
  // depth loop): 204 -> 198 ms of downdates per 20000 x 16000 factorisation
  // at b = 256, where 256 x 128 tiles (one workgroup per CU, nothing to
  // hide the epilogue behind) took 217 ms.
  const bool deep = K >= 192 && cdiv(M, Big::BM) * cdiv(N, Big::BN) >= 4 * kNumCU;
  const int64_t tiles = deep ? cdiv(M, Big::BM) * cdiv(N, Big::BN)
                             : cdiv(M, Small::BM) * cdiv(N, Small::BN);
  if (tiles > INT32_MAX - 8) return kEInval;
  const dim3 grid(static_cast<unsigned>(8 * cdiv(tiles, 8)));  // dd_tile
  {
    ProfScope ps(kKDowndate, 2.0 * M * N * K, 8.0 * (2 * M * N + M * K + K * N), s);
    const int vr = vec_ok(R, ldr), vab = vec_ok(Qm, ldq) & vec_ok(B, ldb);
    if (deep)
      hipLaunchKernelGGL((downdate_kernel<Big, false>), grid, dim3(Big::NT), 0, s, R, ldr, Qm,
                         ldq, B, ldb, M, N, K, sq_part, vr, vab);
    else
      hipLaunchKernelGGL((downdate_kernel<Small, true>), grid, dim3(Small::NT), 0, s, R, ldr, Qm,
                         ldq, B, ldb, M, N, K, sq_part, vr, vab);
  }
  QB_HIP_TRY(hipGetLastError());
  if (sq_count) *sq_count = static_cast<int>(tiles);
  return kOk;
}

}  // namespace qb
