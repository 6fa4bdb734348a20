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
//   precision 2 (bf16x3):  x = hi + lo with hi = bf16(float(x)),
//                          lo = bf16(float(x) - hi);
//                          x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y on
//                          v_mfma_f32_16x16x32_bf16 (about 2^-16 relative)
//
// Lane layouts (measured on gfx950), both with result element r of lane l
// at D[4 (l / 16) + r][l % 16]:
//   f32 16x16x4    A lane l: A[l % 16][l / 16];   B lane l: B[l / 16][l % 16]
//   bf16 16x16x32  A lane l: A[l % 16][8 (l / 16) + i], i < 8;
//                  B lane l: B[8 (l / 16) + i][l % 16]
//
// Tiles: eight waves of 64 x 64 each, the panel side of the tile covering
// the whole panel so that X (the residual) is read once: Y = X W takes
// 128 x 256 tiles for panels W of 129..256 columns and 256 x 128 for
// narrower ones; C = Q^T X takes 256 x 128 for panels Q of 129..256 columns
// and 128 x 256 for narrower ones.  With 128 x 128 tiles a 256-wide panel read
// the residual twice (counters at 20000 x 16000: 2.15x the algorithmic
// bytes).  Operands move as 16-byte pairs of doubles, are rounded while
// they are written to LDS, and two LDS stages let the next depth slice be
// loaded and stored while the current one is multiplied (one barrier per
// slice).
#include "qb_internal.hpp"

namespace qb {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));

template <int PREC>
struct Elem;
template <>
struct Elem<1> {  // f32: 16 depth indices per slice, 18 floats per LDS row
  static constexpr int BK = 16, SK = 18;
};
template <>
struct Elem<2> {  // bf16x3: 32 depth indices per slice, 40 bf16 (80 bytes) per LDS row
  static constexpr int BK = 32, SK = 40;
};

template <int PREC, int BM_, int BN_, int WGM_, int WGN_>
struct LShape {
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WM = BM / WGM, WN = BN / WGN, IB = WM / 16, JB = WN / 16;
  static constexpr int BK = Elem<PREC>::BK, SK = Elem<PREC>::SK;
  // double pairs per thread per slice, of A (BM x BK) and of B (BN x BK)
  static constexpr int PA = BM * BK / (2 * NT), PB = BN * BK / (2 * NT);
  // LDS bytes of one stage: f32 A, B; bf16x3 A hi, A lo, B hi, B lo
  static constexpr int STAGE = PREC == 1 ? (BM + BN) * SK * 4 : 2 * (BM + BN) * SK * 2;
  static_assert(PA >= 1 && PB >= 1 && PA * 2 * NT == BM * BK && PB * 2 * NT == BN * BK,
                "whole pairs per thread");
  static_assert(WM == 64 && WN == 64, "64 x 64 per wave");
};
template <int PREC>
using NNS = LShape<PREC, 128, 256, 2, 4>;
template <int PREC>
using TNS = LShape<PREC, 256, 128, 4, 2>;

__device__ __forceinline__ double2 ld_pair(const double* p, bool ok0, bool ok1, bool vec) {
  if (vec && ok0 && ok1) return *reinterpret_cast<const double2*>(p);
  double2 v = make_double2(0.0, 0.0);
  if (ok0) v.x = p[0];
  if (ok1) v.y = p[1];
  return v;
}

// x ~ hi + lo to about 2^-17 relative: x rounded to float (xf), hi = xf
// rounded to bf16, lo = the exact float difference xf - hi rounded to bf16.
// xf is kept opaque so that each rounding to bf16 is one packed conversion
// (v_cvt_pk_bf16_f32): written as bf16(float(x)) the compiler emits a
// correctly rounded double -> bf16 sequence of about twelve instructions,
// and the double-precision lo about fourteen more (counters: the bf16x3
// sample spent about 45 % of its cycles on VALU work).
__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  float xf = static_cast<float>(x);
  asm volatile("" : "+v"(xf));
  hi = static_cast<__bf16>(xf);
  lo = static_cast<__bf16>(xf - static_cast<float>(hi));
}

// Accumulate the BM x BN tile over k in [kbeg, kend).  A is M x K, element
// (m, k) at A[m + k lda] (m-contiguous) or A[k + m lda] (A_KCONTIG); B is
// K x N, element (k, n) at B[k + n ldb].  vec: both operands allow 16-byte
// pair loads (16-byte aligned base, even ld).
template <int PREC, class S, bool A_KCONTIG>
__device__ __forceinline__ void lowp_loop(const double* __restrict__ A, int64_t lda,
                                          const double* __restrict__ Bm, int64_t ldb, int64_t m0,
                                          int64_t n0, int64_t M, int64_t N, int64_t kbeg,
                                          int64_t kend, bool vec, char* smem,
                                          f4 (&acc)[S::IB][S::JB]) {
  constexpr int BK = S::BK, SK = S::SK, NT = S::NT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave % S::WGM) * S::WM, wn = (wave / S::WGM) * S::WN;
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  if (kbeg >= kend) return;

  double2 ra[S::PA], rb[S::PB];
  auto gload = [&](int64_t kc) {
#pragma unroll
    for (int q = 0; q < S::PA; ++q) {
      const int e = t + NT * q;
      if (A_KCONTIG) {  // pair (row r, depth 2 kp .. 2 kp + 1)
        const int kp = e % (BK / 2), r = e / (BK / 2);
        const int64_t gm = m0 + r, gk = kc + 2 * kp;
        ra[q] = ld_pair(A + gk + gm * lda, gm < M && gk < kend, gm < M && gk + 1 < kend, vec);
      } else {          // pair (rows 2 rp .. 2 rp + 1, depth kk)
        const int rp = e % (S::BM / 2), kk = e / (S::BM / 2);
        const int64_t gm = m0 + 2 * rp, gk = kc + kk;
        ra[q] = ld_pair(A + gm + gk * lda, gm < M && gk < kend, gm + 1 < M && gk < kend, vec);
      }
    }
#pragma unroll
    for (int q = 0; q < S::PB; ++q) {
      const int e = t + NT * q;
      const int kp = e % (BK / 2), c = e / (BK / 2);
      const int64_t gn = n0 + c, gk = kc + 2 * kp;
      rb[q] = ld_pair(Bm + gk + gn * ldb, gn < N && gk < kend, gn < N && gk + 1 < kend, vec);
    }
  };

  if constexpr (PREC == 1) {
    auto sstore = [&](int stage) {
      float* As = reinterpret_cast<float*>(smem + stage * S::STAGE);
      float* Bs = As + S::BM * SK;
#pragma unroll
      for (int q = 0; q < S::PA; ++q) {
        const int e = t + NT * q;
        if (A_KCONTIG) {
          const int kp = e % (BK / 2), r = e / (BK / 2);
          *reinterpret_cast<fl2*>(As + r * SK + 2 * kp) =
              (fl2){static_cast<float>(ra[q].x), static_cast<float>(ra[q].y)};
        } else {
          const int rp = e % (S::BM / 2), kk = e / (S::BM / 2);
          As[(2 * rp) * SK + kk] = static_cast<float>(ra[q].x);
          As[(2 * rp + 1) * SK + kk] = static_cast<float>(ra[q].y);
        }
      }
#pragma unroll
      for (int q = 0; q < S::PB; ++q) {
        const int e = t + NT * q;
        const int kp = e % (BK / 2), c = e / (BK / 2);
        *reinterpret_cast<fl2*>(Bs + c * SK + 2 * kp) =
            (fl2){static_cast<float>(rb[q].x), static_cast<float>(rb[q].y)};
      }
    };
    auto compute = [&](int stage) {
      const float* As = reinterpret_cast<const float*>(smem + stage * S::STAGE);
      const float* Bs = As + S::BM * SK;
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kq = 4 * k4 + (lane >> 4);
        float a[S::IB], b[S::JB];
#pragma unroll
        for (int i = 0; i < S::IB; ++i) a[i] = As[(wm + 16 * i + (lane & 15)) * SK + kq];
#pragma unroll
        for (int j = 0; j < S::JB; ++j) b[j] = Bs[(wn + 16 * j + (lane & 15)) * SK + kq];
#pragma unroll
        for (int i = 0; i < S::IB; ++i)
#pragma unroll
          for (int j = 0; j < S::JB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    };
    gload(kbeg);
    sstore(0);
    __syncthreads();
    int stage = 0;
    for (int64_t kc = kbeg; kc < kend; kc += BK) {
      const bool more = kc + BK < kend;
      if (more) gload(kc + BK);
      compute(stage);
      if (more) sstore(stage ^ 1);
      __syncthreads();
      stage ^= 1;
    }
  } else {
    auto sstore = [&](int stage) {
      __bf16* Ah = reinterpret_cast<__bf16*>(smem + stage * S::STAGE);
      __bf16* Al = Ah + S::BM * SK;
      __bf16* Bh = Al + S::BM * SK;
      __bf16* Bl = Bh + S::BN * SK;
#pragma unroll
      for (int q = 0; q < S::PA; ++q) {
        const int e = t + NT * q;
        __bf16 h0, l0, h1, l1;
        split_bf16(ra[q].x, h0, l0);
        split_bf16(ra[q].y, h1, l1);
        if (A_KCONTIG) {
          const int kp = e % (BK / 2), r = e / (BK / 2);
          *reinterpret_cast<bf2*>(Ah + r * SK + 2 * kp) = (bf2){h0, h1};
          *reinterpret_cast<bf2*>(Al + r * SK + 2 * kp) = (bf2){l0, l1};
        } else {
          const int rp = e % (S::BM / 2), kk = e / (S::BM / 2);
          Ah[(2 * rp) * SK + kk] = h0;
          Al[(2 * rp) * SK + kk] = l0;
          Ah[(2 * rp + 1) * SK + kk] = h1;
          Al[(2 * rp + 1) * SK + kk] = l1;
        }
      }
#pragma unroll
      for (int q = 0; q < S::PB; ++q) {
        const int e = t + NT * q;
        const int kp = e % (BK / 2), c = e / (BK / 2);
        __bf16 h0, l0, h1, l1;
        split_bf16(rb[q].x, h0, l0);
        split_bf16(rb[q].y, h1, l1);
        *reinterpret_cast<bf2*>(Bh + c * SK + 2 * kp) = (bf2){h0, h1};
        *reinterpret_cast<bf2*>(Bl + c * SK + 2 * kp) = (bf2){l0, l1};
      }
    };
    auto compute = [&](int stage) {
      const __bf16* Ah = reinterpret_cast<const __bf16*>(smem + stage * S::STAGE);
      const __bf16* Al = Ah + S::BM * SK;
      const __bf16* Bh = Al + S::BM * SK;
      const __bf16* Bl = Bh + S::BN * SK;
      const int k8 = 8 * (lane >> 4);
      bf8 bh[S::JB], bl[S::JB];
#pragma unroll
      for (int j = 0; j < S::JB; ++j) {
        const int col = wn + 16 * j + (lane & 15);
        bh[j] = *reinterpret_cast<const bf8*>(Bh + col * SK + k8);
        bl[j] = *reinterpret_cast<const bf8*>(Bl + col * SK + k8);
      }
#pragma unroll
      for (int i = 0; i < S::IB; ++i) {
        const int row = wm + 16 * i + (lane & 15);
        const bf8 ah = *reinterpret_cast<const bf8*>(Ah + row * SK + k8);
        const bf8 al = *reinterpret_cast<const bf8*>(Al + row * SK + k8);
#pragma unroll
        for (int j = 0; j < S::JB; ++j) {
          // small terms first so they are not absorbed by the large one
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
        }
      }
    };
    gload(kbeg);
    sstore(0);
    __syncthreads();
    int stage = 0;
    for (int64_t kc = kbeg; kc < kend; kc += BK) {
      const bool more = kc + BK < kend;
      if (more) gload(kc + BK);
      compute(stage);
      if (more) sstore(stage ^ 1);
      __syncthreads();
      stage ^= 1;
    }
  }
}

// out tile -> partial buffer part[z] (M x N, ld = M) or, when part is null,
// directly to out (ld, optional transposed store)
template <class S>
__device__ __forceinline__ void store_tile(const f4 (&acc)[S::IB][S::JB], int64_t m0, int64_t n0,
                                           int64_t M, int64_t N, double* __restrict__ part,
                                           double* __restrict__ out, int64_t ldo, int transpose) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave % S::WGM) * S::WM, wn = (wave / S::WGM) * S::WN;
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t col = n0 + wn + 16 * j + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (row < M && col < N) {
          const double v = static_cast<double>(acc[i][j][r]);
          if (part != nullptr) part[static_cast<int64_t>(blockIdx.z) * M * N + row + col * M] = v;
          else if (transpose) out[col + row * ldo] = v;
          else out[row + col * ldo] = v;
        }
      }
    }
}

// Y = X W (X m-contiguous).  grid (M tiles, N tiles, split).
template <int PREC, class S>
__global__ __launch_bounds__(S::NT, 1) void lowp_nn_kernel(
    const double* __restrict__ X, int64_t ldx, const double* __restrict__ W, int64_t ldw,
    double* __restrict__ Y, int64_t ldy, int64_t M, int64_t N, int64_t K, int64_t kchunk,
    int vec, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char smem[2 * S::STAGE];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * S::BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * S::BN;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  f4 acc[S::IB][S::JB];
  lowp_loop<PREC, S, false>(X, ldx, W, ldw, m0, n0, M, N, kbeg, kend, vec != 0, smem, acc);
  store_tile<S>(acc, m0, n0, M, N, part, Y, ldy, 0);
}

// C = Q^T X (Q: K x P, so the A operand is k-contiguous).  grid (N tiles,
// P tiles, split)
template <int PREC, class S>
__global__ __launch_bounds__(S::NT, 1) void lowp_tn_kernel(
    const double* __restrict__ Qm, int64_t ldq, const double* __restrict__ X, int64_t ldx,
    double* __restrict__ C, int64_t ldc, int64_t P, int64_t N, int64_t K, int64_t kchunk,
    int transpose, int vec, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char smem[2 * S::STAGE];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * S::BN;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * S::BM;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  f4 acc[S::IB][S::JB];
  lowp_loop<PREC, S, true>(Qm, ldq, X, ldx, m0, n0, P, N, kbeg, kend, vec != 0, smem, acc);
  store_tile<S>(acc, m0, n0, P, N, part, C, ldc, transpose);
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

int pair_ok(const double* p, int64_t ld) {
  return ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && (ld & 1) == 0) ? 1 : 0;
}

template <int PREC, class S>
int nn_impl(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y, int64_t ldy,
            int64_t M, int64_t N, int64_t K, int split, double* part, hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  if (K <= 0) return zero_matrix(Y, ldy, M, N, s);
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? chunk_for(K, split, S::BK) : K;
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(M, S::BM)), static_cast<unsigned>(cdiv(N, S::BN)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmNNLowp, 2.0 * M * N * K * (PREC == 2 ? 3 : 1), 8.0 * (M * K + K * N + M * N), s);
    hipLaunchKernelGGL((lowp_nn_kernel<PREC, S>), grid, dim3(S::NT), 0, s, X, ldx, W, ldw, Y, ldy, M,
                       N, K, kc, pair_ok(X, ldx) & pair_ok(W, ldw),
                       nz > 1 ? part : static_cast<double*>(nullptr));
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

template <int PREC, class S>
int tn_impl(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C, int64_t ldc,
            int64_t P, int64_t N, int64_t K, bool tr, int split, double* part, hipStream_t s) {
  if (P <= 0 || N <= 0) return kOk;
  if (K <= 0) return tr ? zero_matrix(C, ldc, N, P, s) : zero_matrix(C, ldc, P, N, s);
  if (split > 1 && part == nullptr) return kEInval;
  const int64_t kc = split > 1 ? chunk_for(K, split, S::BK) : K;
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(N, S::BN)), static_cast<unsigned>(cdiv(P, S::BM)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmTNLowp, 2.0 * P * N * K * (PREC == 2 ? 3 : 1), 8.0 * (K * P + K * N + P * N), s);
    hipLaunchKernelGGL((lowp_tn_kernel<PREC, S>), grid, dim3(S::NT), 0, s, Qm, ldq, X, ldx, C, ldc, P,
                       N, K, kc, tr ? 1 : 0, pair_ok(Qm, ldq) & pair_ok(X, ldx),
                       nz > 1 ? part : static_cast<double*>(nullptr));
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

int lowp_split(int precision, bool nn, int64_t M, int64_t N, int64_t K) {
  // one eight-wave workgroup per CU in both precisions (bf16x3: two 61 KB
  // LDS stages; f32: about 145 VGPRs, so two waves per SIMD)
  (void)precision;
  const bool wide_tile = nn ? N > TNS<1>::BN : M <= NNS<1>::BM;  // 128 x 256
  if (wide_tile) return choose_split_fill(M, N, K, 1, NNS<1>::BM, NNS<1>::BN);
  return choose_split_fill(M, N, K, 1, TNS<1>::BM, TNS<1>::BN);
}

int gemm_nn_lowp(int precision, const double* X, int64_t ldx, const double* W, int64_t ldw,
                 double* Y, int64_t ldy, int64_t M, int64_t N, int64_t K, int split,
                 double* part, hipStream_t s) {
  // panels up to 128 wide take 256 x 128 tiles (a 128 x 256 tile would
  // multiply half a tile of zeros)
  const bool narrow = N <= TNS<1>::BN;
  if (precision == 1)
    return narrow ? nn_impl<1, TNS<1>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, part, s)
                  : nn_impl<1, NNS<1>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, part, s);
  if (precision == 2)
    return narrow ? nn_impl<2, TNS<2>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, part, s)
                  : nn_impl<2, NNS<2>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, part, s);
  return kEInval;
}

int gemm_tn_lowp(int precision, const double* Qm, int64_t ldq, const double* X, int64_t ldx,
                 double* C, int64_t ldc, int64_t P, int64_t N, int64_t K, bool transpose_out,
                 int split, double* part, hipStream_t s) {
  // panels Q up to 128 wide take 128 x 256 tiles (a 256-row tile would
  // multiply half a tile of zeros)
  const bool narrow = P <= NNS<1>::BM;
  if (precision == 1)
    return narrow ? tn_impl<1, NNS<1>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, part, s)
                  : tn_impl<1, TNS<1>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, part, s);
  if (precision == 2)
    return narrow ? tn_impl<2, NNS<2>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, part, s)
                  : tn_impl<2, TNS<2>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, part, s);
  return kEInval;
}

}  // namespace qb
