// Mixed-precision sampling products for the blocked QB (gfx950).
//
// The sampling products of Figure 4 step (3) and Figure 6 steps (5)-(6)
// (A Omega, A^T Q, A Z) only choose the subspace; the residual is always
// downdated and measured in float64, so an error in a sample costs rank,
// never accuracy of the final factorisation.  These kernels read the float64
// operands from HBM, round them on the way into LDS, multiply on the MFMA
// units and accumulate in float32; results are returned in float64.
//
//   precision 1 (f32):     v_mfma_f32_16x16x4_f32 on operands rounded to
//                          float32 (relative error about 2^-24 per term)
//   precision 2 (bf16x3):  x = hi + lo with hi = bf16(x), lo = bf16(x - hi);
//                          x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y on
//                          v_mfma_f32_16x16x32_bf16 (about 2^-16 relative)
//
// Lane layouts (measured on gfx950), both with result element r of lane l
// at D[4 (l / 16) + r][l % 16]:
//   f32 16x16x4    A lane l: A[l % 16][l / 16];   B lane l: B[l / 16][l % 16]
//   bf16 16x16x32  A lane l: A[l % 16][8 (l / 16) + i], i < 8;
//                  B lane l: B[8 (l / 16) + i][l % 16]
#include "qb_internal.hpp"

namespace qb {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128, NT = 256;

template <int PREC>
struct Cfg;
template <>
struct Cfg<1> {  // f32
  static constexpr int BK = 16;
  static constexpr int SK = BK + 1;  // floats per LDS row (k contiguous)
};
template <>
struct Cfg<2> {  // bf16x3
  static constexpr int BK = 32;
  static constexpr int SK = 40;      // bf16 per LDS row: 80-byte stride
};

// global operand (m, k) element address helper
template <bool KCONTIG>
__device__ __forceinline__ double load_op(const double* __restrict__ X, int64_t ld, int64_t r,
                                          int64_t kk, bool ok) {
  if (!ok) return 0.0;
  return KCONTIG ? X[kk + r * ld] : X[r + kk * ld];
}

// C tile (BM x BN) accumulated over k in [kbeg, kend); A is M x K (m- or
// k-contiguous in global memory), B is K x N with k contiguous.
template <int PREC, bool A_KCONTIG>
__device__ __forceinline__ void lowp_loop(const double* __restrict__ A, int64_t lda,
                                          const double* __restrict__ Bm, int64_t ldb, int64_t m0,
                                          int64_t n0, int64_t M, int64_t N, int64_t kbeg,
                                          int64_t kend, char* smem, f4 acc[4][4]) {
  constexpr int BK = Cfg<PREC>::BK, SK = Cfg<PREC>::SK;
  constexpr int PER = (BM * BK) / NT;  // elements of each operand per thread per fill
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  if (kbeg >= kend) return;

  double ra[PER], rb[PER];
  auto gload = [&](int64_t kc) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = t + NT * q;
      int mi, ki;
      if (A_KCONTIG) { ki = e % BK; mi = e / BK; } else { mi = e % BM; ki = e / BM; }
      const int64_t gm = m0 + mi, gk = kc + ki;
      ra[q] = load_op<A_KCONTIG>(A, lda, gm, gk, gm < M && gk < kend);
      const int kb = e % BK, nb = e / BK;
      const int64_t gn = n0 + nb, gkb = kc + kb;
      rb[q] = load_op<true>(Bm, ldb, gn, gkb, gn < N && gkb < kend);
    }
  };

  if constexpr (PREC == 1) {
    float* As = reinterpret_cast<float*>(smem);
    float* Bs = As + BM * SK;
    auto sstore = [&]() {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = t + NT * q;
        int mi, ki;
        if (A_KCONTIG) { ki = e % BK; mi = e / BK; } else { mi = e % BM; ki = e / BM; }
        As[mi * SK + ki] = static_cast<float>(ra[q]);
        Bs[(e / BK) * SK + (e % BK)] = static_cast<float>(rb[q]);
      }
    };
    gload(kbeg);
    sstore();
    __syncthreads();
    for (int64_t kc = kbeg; kc < kend; kc += BK) {
      const bool more = kc + BK < kend;
      if (more) gload(kc + BK);
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kq = 4 * k4 + (lane >> 4);
        float a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[(wm + 16 * i + (lane & 15)) * SK + kq];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[(wn + 16 * j + (lane & 15)) * SK + kq];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
      if (more) {
        sstore();
        __syncthreads();
      }
    }
  } else {
    __bf16* Ah = reinterpret_cast<__bf16*>(smem);
    __bf16* Al = Ah + BM * SK;
    __bf16* Bh = Al + BM * SK;
    __bf16* Bl = Bh + BN * SK;
    auto sstore = [&]() {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = t + NT * q;
        int mi, ki;
        if (A_KCONTIG) { ki = e % BK; mi = e / BK; } else { mi = e % BM; ki = e / BM; }
        const __bf16 ah = static_cast<__bf16>(static_cast<float>(ra[q]));
        const __bf16 al = static_cast<__bf16>(static_cast<float>(ra[q] - static_cast<double>(static_cast<float>(ah))));
        Ah[mi * SK + ki] = ah;
        Al[mi * SK + ki] = al;
        const __bf16 bh = static_cast<__bf16>(static_cast<float>(rb[q]));
        const __bf16 bl = static_cast<__bf16>(static_cast<float>(rb[q] - static_cast<double>(static_cast<float>(bh))));
        const int o = (e / BK) * SK + (e % BK);
        Bh[o] = bh;
        Bl[o] = bl;
      }
    };
    gload(kbeg);
    sstore();
    __syncthreads();
    for (int64_t kc = kbeg; kc < kend; kc += BK) {
      const bool more = kc + BK < kend;
      if (more) gload(kc + BK);
      const int k8 = 8 * (lane >> 4);
      bf8 bh[4], bl[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = wn + 16 * j + (lane & 15);
        bh[j] = *reinterpret_cast<const bf8*>(Bh + col * SK + k8);
        bl[j] = *reinterpret_cast<const bf8*>(Bl + col * SK + k8);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm + 16 * i + (lane & 15);
        const bf8 ah = *reinterpret_cast<const bf8*>(Ah + row * SK + k8);
        const bf8 al = *reinterpret_cast<const bf8*>(Al + row * SK + k8);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // small terms first so they are not absorbed by the large one
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
        }
      }
      __syncthreads();
      if (more) {
        sstore();
        __syncthreads();
      }
    }
  }
}

template <int PREC>
constexpr int smem_bytes() {
  return PREC == 1 ? (BM + BN) * Cfg<1>::SK * 4 : 2 * (BM + BN) * Cfg<2>::SK * 2;
}

__device__ __forceinline__ int acc_row(int i, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 64 + 16 * i + 4 * (lane >> 4) + r;
}
__device__ __forceinline__ int acc_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 64 + 16 * j + (lane & 15);
}

// out tile -> partial buffer part[z] (rows x cols, ld = rows) or, when
// part is null, directly to out (ld, optional transposed store)
__device__ __forceinline__ void store_tile(const f4 acc[4][4], int64_t m0, int64_t n0, int64_t M,
                                           int64_t N, double* __restrict__ part,
                                           double* __restrict__ out, int64_t ldo, int transpose) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + acc_col(j);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + acc_row(i, r);
        if (row < M && col < N) {
          const double v = static_cast<double>(acc[i][j][r]);
          if (part != nullptr) part[static_cast<int64_t>(blockIdx.z) * M * N + row + col * M] = v;
          else if (transpose) out[col + row * ldo] = v;
          else out[row + col * ldo] = v;
        }
      }
    }
}

// Y = X W (X m-contiguous).  grid (M tiles, N tiles, split).  The bf16x3
// form holds 32 prefetched doubles per thread and runs one workgroup per CU.
template <int PREC>
__global__ __launch_bounds__(NT, PREC == 2 ? 1 : 2) void lowp_nn_kernel(const double* __restrict__ X, int64_t ldx,
                                                        const double* __restrict__ W, int64_t ldw,
                                                        double* __restrict__ Y, int64_t ldy,
                                                        int64_t M, int64_t N, int64_t K,
                                                        int64_t kchunk, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<PREC>()];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * BN;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  f4 acc[4][4];
  lowp_loop<PREC, false>(X, ldx, W, ldw, m0, n0, M, N, kbeg, kend, smem, acc);
  store_tile(acc, m0, n0, M, N, part, Y, ldy, 0);
}

// C = Q^T X (Q: K x P, so the A operand is k-contiguous).  grid (N tiles, P tiles, split)
template <int PREC>
__global__ __launch_bounds__(NT, 2) void lowp_tn_kernel(const double* __restrict__ Qm, int64_t ldq,
                                                        const double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ C, int64_t ldc,
                                                        int64_t P, int64_t N, int64_t K,
                                                        int64_t kchunk, int transpose,
                                                        double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char smem[smem_bytes<PREC>()];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * BN;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * BM;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  f4 acc[4][4];
  lowp_loop<PREC, true>(Qm, ldq, X, ldx, m0, n0, P, N, kbeg, kend, smem, acc);
  store_tile(acc, m0, n0, P, N, part, C, ldc, transpose);
}

// out = sum_s part[s] (fixed order), optional transposed store
__global__ __launch_bounds__(256) void lowp_reduce_kernel(const double* __restrict__ part,
                                                          int split, double* __restrict__ out,
                                                          int64_t ldo, int64_t M, int64_t N,
                                                          int transpose) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = M * N;
  if (idx >= total) return;
  double s = 0.0;
  for (int z = 0; z < split; ++z) s += part[static_cast<int64_t>(z) * total + idx];
  const int64_t i = idx % M, j = idx / M;
  out[transpose ? (j + i * ldo) : (i + j * ldo)] = s;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t chunk_for(int64_t K, int split, int bk) {
  const int64_t c = cdiv(K, split);
  return cdiv(c, bk) * bk;
}

template <int PREC>
int nn_impl(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y, int64_t ldy,
            int64_t M, int64_t N, int64_t K, int split, double* part, hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  if (K <= 0) return zero_matrix(Y, ldy, M, N, s);
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? chunk_for(K, split, Cfg<PREC>::BK) : K;
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(M, BM)), static_cast<unsigned>(cdiv(N, BN)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmNNLowp, 2.0 * M * N * K * (PREC == 2 ? 3 : 1), 8.0 * (M * K + K * N + M * N), s);
    hipLaunchKernelGGL(lowp_nn_kernel<PREC>, grid, dim3(NT), 0, s, X, ldx, W, ldw, Y, ldy, M, N,
                       K, kc, nz > 1 ? part : static_cast<double*>(nullptr));
  }
  QB_HIP_TRY(hipGetLastError());
  if (nz > 1) {
    const int64_t total = M * N;
    ProfScope ps(kKReduce, double(nz) * total, 8.0 * (nz + 1) * total, s);
    hipLaunchKernelGGL(lowp_reduce_kernel, dim3(static_cast<unsigned>(cdiv(total, 256))), dim3(256),
                       0, s, part, nz, Y, ldy, M, N, 0);
    QB_HIP_TRY(hipGetLastError());
  }
  return kOk;
}

template <int PREC>
int tn_impl(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C, int64_t ldc,
            int64_t P, int64_t N, int64_t K, bool tr, int split, double* part, hipStream_t s) {
  if (P <= 0 || N <= 0) return kOk;
  if (K <= 0) return tr ? zero_matrix(C, ldc, N, P, s) : zero_matrix(C, ldc, P, N, s);
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? chunk_for(K, split, Cfg<PREC>::BK) : K;
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(N, BN)), static_cast<unsigned>(cdiv(P, BM)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmTNLowp, 2.0 * P * N * K * (PREC == 2 ? 3 : 1), 8.0 * (K * P + K * N + P * N), s);
    hipLaunchKernelGGL(lowp_tn_kernel<PREC>, grid, dim3(NT), 0, s, Qm, ldq, X, ldx, C, ldc, P, N,
                       K, kc, tr ? 1 : 0, nz > 1 ? part : static_cast<double*>(nullptr));
  }
  QB_HIP_TRY(hipGetLastError());
  if (nz > 1) {
    const int64_t total = P * N;
    ProfScope ps(kKReduce, double(nz) * total, 8.0 * (nz + 1) * total, s);
    hipLaunchKernelGGL(lowp_reduce_kernel, dim3(static_cast<unsigned>(cdiv(total, 256))), dim3(256),
                       0, s, part, nz, C, ldc, P, N, tr ? 1 : 0);
    QB_HIP_TRY(hipGetLastError());
  }
  return kOk;
}

}  // namespace

int gemm_nn_lowp(int precision, const double* X, int64_t ldx, const double* W, int64_t ldw,
                 double* Y, int64_t ldy, int64_t M, int64_t N, int64_t K, int split,
                 double* part, hipStream_t s) {
  if (precision == 1) return nn_impl<1>(X, ldx, W, ldw, Y, ldy, M, N, K, split, part, s);
  if (precision == 2) return nn_impl<2>(X, ldx, W, ldw, Y, ldy, M, N, K, split, part, s);
  return kEInval;
}

int gemm_tn_lowp(int precision, const double* Qm, int64_t ldq, const double* X, int64_t ldx,
                 double* C, int64_t ldc, int64_t P, int64_t N, int64_t K, bool transpose_out,
                 int split, double* part, hipStream_t s) {
  if (precision == 1)
    return tn_impl<1>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, part, s);
  if (precision == 2)
    return tn_impl<2>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, part, s);
  return kEInval;
}

}  // namespace qb
