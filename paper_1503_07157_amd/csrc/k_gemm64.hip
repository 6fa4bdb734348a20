// FP64 MFMA GEMM kernels of the blocked QB hot path (gfx950).
//
// Every product of Figure 4 / Figure 6 has one long side and one side of at
// most b (<= 256) columns:
//   gemm_nn   Y = X W            A Omega_i, A Z, Qbar C, Y T^{-1}   (K = long or b)
//   gemm_tn   C = Q^T X          Q_i^T A, Q_i^T Qbar, Y^T Y         (K = m, long)
//   downdate  R = R - Q_i B_i    with the fused residual sum of squares
// A workgroup of 256 threads (4 waves) owns a 128 x 128 output tile; each
// wave owns a 64 x 64 sub-tile as 4 x 4 blocks of v_mfma_f64_16x16x4_f64.
// Operand tiles of depth 16 are staged through LDS with register
// prefetch of the next depth slice.  Long reductions are split over
// workgroups (split-K) into partial buffers that a second kernel sums in a
// fixed order, so results are bitwise reproducible run to run.
//
// MFMA f64 16x16x4 lane layout (measured on gfx950):
//   A operand  lane l holds A[l % 16][l / 16]        (16 x 4)
//   B operand  lane l holds B[l / 16][l % 16]        (4 x 16)
//   result     lane l, element r holds D[l / 16 + 4 r][l % 16]
#include "qb_internal.hpp"

namespace qb {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = kTileM, BN = kTileN, BK = kTileK, NT = kGemmThreads;
constexpr int SA_M = BM + 1;  // A stored [k][m] (m contiguous)
constexpr int SA_K = BK + 1;  // A stored [m][k] (k contiguous)
constexpr int SB_K = BK + 1;  // B stored [n][k] (k contiguous)
constexpr int A_LDS = (BK * SA_M > BM * SA_K) ? BK * SA_M : BM * SA_K;
constexpr int B_LDS = BN * SB_K;
constexpr int PER_THREAD = (BM * BK) / NT;  // 8 elements of each operand per fill

// A is "m-contiguous" when its global layout has consecutive rows adjacent
// (X column-major, element (m, k) at X[m + k*ld]); "k-contiguous" when
// element (m, k) lies at X[k + m*ld] (the transposed operand Q^T).
template <bool A_KCONTIG>
struct Tile {
  double ra[PER_THREAD];
  double rb[PER_THREAD];

  __device__ __forceinline__ void load(const double* __restrict__ A, int64_t lda,
                                       const double* __restrict__ Bm, int64_t ldb, int64_t m0,
                                       int64_t n0, int64_t M, int64_t N, int64_t kc,
                                       int64_t kend) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER_THREAD; ++q) {
      const int e = t + NT * q;
      if (A_KCONTIG) {
        const int kk = e % BK, i = e / BK;
        const int64_t gm = m0 + i, gk = kc + kk;
        ra[q] = (gm < M && gk < kend) ? A[gk + gm * lda] : 0.0;
      } else {
        const int row = e % BM, col = e / BM;
        const int64_t gm = m0 + row, gk = kc + col;
        ra[q] = (gm < M && gk < kend) ? A[gm + gk * lda] : 0.0;
      }
      const int kk = e % BK, nn = e / BK;
      const int64_t gn = n0 + nn, gk = kc + kk;
      rb[q] = (gn < N && gk < kend) ? Bm[gk + gn * ldb] : 0.0;
    }
  }

  __device__ __forceinline__ void store(double* As, double* Bs) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER_THREAD; ++q) {
      const int e = t + NT * q;
      if (A_KCONTIG) {
        As[(e / BK) * SA_K + (e % BK)] = ra[q];
      } else {
        As[(e / BM) * SA_M + (e % BM)] = ra[q];
      }
      Bs[(e / BK) * SB_K + (e % BK)] = rb[q];
    }
  }
};

// Accumulate the workgroup tile over k in [kbeg, kend).
template <bool A_KCONTIG>
__device__ __forceinline__ void mma_loop(const double* __restrict__ A, int64_t lda,
                                         const double* __restrict__ Bm, int64_t ldb, int64_t m0,
                                         int64_t n0, int64_t M, int64_t N, int64_t kbeg,
                                         int64_t kend, double* As, double* Bs, d4 acc[4][4]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
  if (kbeg >= kend) return;

  Tile<A_KCONTIG> tl;
  tl.load(A, lda, Bm, ldb, m0, n0, M, N, kbeg, kend);
  tl.store(As, Bs);
  __syncthreads();
  for (int64_t kc = kbeg; kc < kend; kc += BK) {
    const bool more = kc + BK < kend;
    if (more) tl.load(A, lda, Bm, ldb, m0, n0, M, N, kc + BK, kend);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      double a[4], b[4];
      const int kq = 4 * k4 + lk;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int mrow = wm + 16 * i + lr;
        a[i] = A_KCONTIG ? As[mrow * SA_K + kq] : As[kq * SA_M + mrow];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[(wn + 16 * j + lr) * SB_K + kq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      tl.store(As, Bs);
      __syncthreads();
    }
  }
}

// row / column of accumulator element (i, j, r) inside the workgroup tile
__device__ __forceinline__ int acc_row(int i, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 64 + 16 * i + (lane >> 4) + 4 * r;
}
__device__ __forceinline__ int acc_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 64 + 16 * j + (lane & 15);
}

// deterministic workgroup sum; every thread passes its value, thread 0
// returns the total
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) tot += red[w];
  return tot;
}

// ---------------------------------------------------------------------------
// Y = alpha X W + beta Y   (X: M x K m-contiguous, W: K x N, k-contiguous)
// grid: (M tiles, N tiles, split); split > 1 writes part[z][M x N]
__global__ __launch_bounds__(NT, 2) void gemm_nn_kernel(const double* __restrict__ X, int64_t ldx,
                                                        const double* __restrict__ W, int64_t ldw,
                                                        double* __restrict__ Y, int64_t ldy,
                                                        int64_t M, int64_t N, int64_t K,
                                                        int64_t kchunk, double alpha, double beta,
                                                        double* __restrict__ part) {
  __shared__ double As[A_LDS];
  __shared__ double Bs[B_LDS];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * BN;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  d4 acc[4][4];
  mma_loop<false>(X, ldx, W, ldw, m0, n0, M, N, kbeg, kend, As, Bs, acc);
  if (part != nullptr) {
    double* P = part + static_cast<int64_t>(blockIdx.z) * M * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = n0 + acc_col(j);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + acc_row(i, r);
          if (row < M && col < N) P[row + col * M] = acc[i][j][r];
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = n0 + acc_col(j);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + acc_row(i, r);
          if (row < M && col < N) {
            double v = alpha * acc[i][j][r];
            if (beta != 0.0) v += beta * Y[row + col * ldy];
            Y[row + col * ldy] = v;
          }
        }
      }
  }
}

// C = Q^T X  (Q: K x P so A = Q^T is k-contiguous; X: K x N)
// grid: (N tiles, P tiles, split)
__global__ __launch_bounds__(NT, 2) void gemm_tn_kernel(const double* __restrict__ Qm, int64_t ldq,
                                                        const double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ C, int64_t ldc,
                                                        int64_t P, int64_t N, int64_t K,
                                                        int64_t kchunk, int transpose_out,
                                                        double* __restrict__ part,
                                                        double* __restrict__ sq_part) {
  __shared__ double As[A_LDS];
  __shared__ double Bs[B_LDS];
  __shared__ double red[NT / 64];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * BN;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * BM;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  d4 acc[4][4];
  mma_loop<true>(Qm, ldq, X, ldx, m0, n0, P, N, kbeg, kend, As, Bs, acc);
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + acc_col(j);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + acc_row(i, r);
        if (row < P && col < N) {
          const double v = acc[i][j][r];
          if (part != nullptr) {
            part[static_cast<int64_t>(blockIdx.z) * P * N + row + col * P] = v;
          } else {
            if (transpose_out) C[col + row * ldc] = v; else C[row + col * ldc] = v;
            sq += v * v;
          }
        }
      }
    }
  if (part == nullptr && sq_part != nullptr) {
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) sq_part[blockIdx.x + static_cast<int64_t>(blockIdx.y) * gridDim.x] = tot;
  }
}

// out(M x N) = alpha * sum_s part[s] + beta * out; transposed store puts
// element (i, j) at out[j + i*ldo].  Optional per-block sums of squares.
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int split,
                                                     double* __restrict__ out, int64_t ldo,
                                                     int64_t M, int64_t N, double alpha,
                                                     double beta, int transpose_out,
                                                     double* __restrict__ sq_part) {
  __shared__ double red[4];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = M * N;
  double sq = 0.0;
  if (idx < total) {
    double s = 0.0;
    for (int z = 0; z < split; ++z) s += part[static_cast<int64_t>(z) * total + idx];
    const int64_t i = idx % M, j = idx / M;
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

// R -= Q B; per-workgroup sum of squares of the updated tile.
// grid: (M tiles, N tiles)
__global__ __launch_bounds__(NT, 2) void downdate_kernel(double* __restrict__ R, int64_t ldr,
                                                         const double* __restrict__ Qm,
                                                         int64_t ldq,
                                                         const double* __restrict__ B,
                                                         int64_t ldb, int64_t M, int64_t N,
                                                         int64_t K,
                                                         double* __restrict__ sq_part) {
  __shared__ double As[A_LDS];
  __shared__ double Bs[B_LDS];
  __shared__ double red[NT / 64];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * BN;
  d4 acc[4][4];
  mma_loop<false>(Qm, ldq, B, ldb, m0, n0, M, N, 0, K, As, Bs, acc);
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + acc_col(j);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + acc_row(i, r);
        if (row < M && col < N) {
          const double v = R[row + col * ldr] - acc[i][j][r];
          R[row + col * ldr] = v;
          sq += v * v;
        }
      }
    }
  const double tot = block_sum(sq, red);
  if (threadIdx.x == 0) sq_part[blockIdx.x + static_cast<int64_t>(blockIdx.y) * gridDim.x] = tot;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int choose_split(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = cdiv(M, BM) * cdiv(N, BN);
  int64_t s = cdiv(kSplitTargetWG, tiles > 0 ? tiles : 1);
  const int64_t by_depth = K / kSplitMinDepth;
  if (s > by_depth) s = by_depth;
  const int64_t by_mem = kPartialCapDoubles / ((M * N > 0) ? M * N : 1);
  if (s > by_mem) s = by_mem;
  if (s > kMaxSplit) s = kMaxSplit;
  if (s < 1) s = 1;
  return static_cast<int>(s);
}

size_t partial_doubles(int64_t M, int64_t N, int split) {
  return split > 1 ? static_cast<size_t>(M) * N * split : 0;
}

static int64_t kchunk_for(int64_t K, int split) {
  int64_t c = cdiv(K, split);
  return cdiv(c, BK) * BK;
}

int gemm_nn(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y, int64_t ldy,
            int64_t M, int64_t N, int64_t K, double alpha, double beta, int split, double* part,
            hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  if (K <= 0) split = 1;
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? kchunk_for(K, split) : (K > 0 ? K : 0);
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(M, BM)), static_cast<unsigned>(cdiv(N, BN)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmNN, 2.0 * M * N * K, 8.0 * (M * K + K * N + M * N * (beta != 0.0 ? 2 : 1)), s);
    hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(NT), 0, s, X, ldx, W, ldw, Y, ldy, M, N, K,
                       kc, alpha, beta, split > 1 ? part : nullptr);
  }
  QB_HIP_TRY(hipGetLastError());
  if (split > 1) {
    const int64_t total = M * N;
    ProfScope ps(kKReduce, double(nz) * total, 8.0 * (nz + (beta != 0.0 ? 2 : 1)) * total, s);
    hipLaunchKernelGGL(reduce_kernel, dim3(static_cast<unsigned>(cdiv(total, 256))), dim3(256), 0,
                       s, part, nz, Y, ldy, M, N, alpha, beta, 0, static_cast<double*>(nullptr));
    QB_HIP_TRY(hipGetLastError());
  }
  return kOk;
}

int gemm_tn(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C, int64_t ldc,
            int64_t P, int64_t N, int64_t K, bool transpose_out, int split, double* part,
            double* sq_part, int* sq_count, hipStream_t s) {
  if (P <= 0 || N <= 0) { if (sq_count) *sq_count = 0; return kOk; }
  if (K <= 0) split = 1;
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? kchunk_for(K, split) : (K > 0 ? K : 0);
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(N, BN)), static_cast<unsigned>(cdiv(P, BM)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmTN, 2.0 * P * N * K, 8.0 * (K * P + K * N + P * N), s);
    hipLaunchKernelGGL(gemm_tn_kernel, grid, dim3(NT), 0, s, Qm, ldq, X, ldx, C, ldc, P, N, K, kc,
                       transpose_out ? 1 : 0, split > 1 ? part : nullptr,
                       split > 1 ? static_cast<double*>(nullptr) : sq_part);
  }
  QB_HIP_TRY(hipGetLastError());
  if (split > 1) {
    const int64_t total = P * N;
    const unsigned nb = static_cast<unsigned>(cdiv(total, 256));
    ProfScope ps(kKReduce, double(nz) * total, 8.0 * (nz + 1) * total, s);
    hipLaunchKernelGGL(reduce_kernel, dim3(nb), dim3(256), 0, s, part, nz, C, ldc, P, N, 1.0, 0.0,
                       transpose_out ? 1 : 0, sq_part);
    QB_HIP_TRY(hipGetLastError());
    if (sq_count) *sq_count = sq_part ? static_cast<int>(nb) : 0;
  } else {
    if (sq_count) *sq_count = sq_part ? static_cast<int>(grid.x * grid.y) : 0;
  }
  return kOk;
}

size_t downdate_partials(int64_t M, int64_t N) {
  return static_cast<size_t>(cdiv(M, BM)) * static_cast<size_t>(cdiv(N, BN));
}

int downdate(double* R, int64_t ldr, const double* Qm, int64_t ldq, const double* B, int64_t ldb,
             int64_t M, int64_t N, int64_t K, double* sq_part, int* sq_count, hipStream_t s) {
  if (M <= 0 || N <= 0) { if (sq_count) *sq_count = 0; return kOk; }
  dim3 grid(static_cast<unsigned>(cdiv(M, BM)), static_cast<unsigned>(cdiv(N, BN)));
  {
    ProfScope ps(kKDowndate, 2.0 * M * N * K, 8.0 * (2 * M * N + M * K + K * N), s);
    hipLaunchKernelGGL(downdate_kernel, grid, dim3(NT), 0, s, R, ldr, Qm, ldq, B, ldb, M, N, K,
                       sq_part);
  }
  QB_HIP_TRY(hipGetLastError());
  if (sq_count) *sq_count = static_cast<int>(grid.x * grid.y);
  return kOk;
}

}  // namespace qb
