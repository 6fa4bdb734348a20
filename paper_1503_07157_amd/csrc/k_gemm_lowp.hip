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
// bytes).
//
// The panel (W, or Q) is read by every tile of the product, so it is rounded
// once, by lowp_pack_kernel, into the format the tiles keep in LDS: per
// depth slice, the tile's panel columns one after another, each holding the
// slice's depth indices (f32 values, or the bf16 hi row and, in a second
// plane, the lo row), zero past the panel's depth and width.  A tile's panel
// slice is then one contiguous block, loaded as 16-byte pieces and stored to
// LDS unchanged: half the bytes of the float64 panel and no rounding work in
// the tiles.  The residual is rounded on its way into LDS: for Y = X W
// (X m-contiguous) each thread loads 4 (f32) or 8 (bf16x3) consecutive depth
// indices of one row, so a row's rounded values go to LDS as one 16-byte
// store per plane; for C = Q^T X (X k-contiguous) as pairs of doubles.  Two
// LDS stages let the next depth slice be loaded and stored while the current
// one is multiplied (one barrier per slice).
#include "qb_internal.hpp"

namespace qb {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));  // one 16-byte piece

template <int PREC>
struct Elem;
template <>
struct Elem<1> {  // f32: 16 depth indices per slice, 20 floats (80 bytes) per LDS row
  static constexpr int BK = 16, SK = 20, VK = 4, PLANES = 1;
};
template <>
struct Elem<2> {  // bf16x3: 32 depth indices per slice, 40 bf16 (80 bytes) per LDS row
  static constexpr int BK = 32, SK = 40, VK = 8, PLANES = 2;
};
// VK: depth indices per 16-byte piece of a rounded row (four pieces per
// slice); PLANES: rounded values per element (f32; bf16 hi and lo).  The
// 80-byte LDS rows keep 16-byte stores aligned, and the 16 rows that one
// MFMA fragment read (or one 16-byte store of 16 lanes) touches fall on
// distinct banks.

template <int PREC, int BM_, int BN_, int WGM_, int WGN_>
struct LShape {
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WM = BM / WGM, WN = BN / WGN, IB = WM / 16, JB = WN / 16;
  static constexpr int BK = Elem<PREC>::BK, SK = Elem<PREC>::SK, VK = Elem<PREC>::VK;
  // LDS bytes of one stage: f32 A, B; bf16x3 A hi, A lo, B hi, B lo
  static constexpr int STAGE = PREC == 1 ? (BM + BN) * SK * 4 : 2 * (BM + BN) * SK * 2;
  static_assert(BK == 4 * VK, "four 16-byte pieces per rounded row");
  static_assert(WM == 64 && WN == 64, "64 x 64 per wave");
};
template <int PREC>
using NNS = LShape<PREC, 128, 256, 2, 4>;
template <int PREC>
using TNS = LShape<PREC, 256, 128, 4, 2>;

// rows of the packed panel: its width rounded up to the panel side of the
// tile (every tile reads whole columns)
inline int64_t round_up(int64_t v, int64_t q) { return (v + q - 1) / q * q; }

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

// VK consecutive values rounded into 16-byte pieces: f32 into h; bf16x3 hi
// into h and lo into l
template <int PREC>
__device__ __forceinline__ void round_piece(const double (&v)[Elem<PREC>::VK], u4& h, u4& l) {
  if constexpr (PREC == 1) {
    const f4 f = (f4){static_cast<float>(v[0]), static_cast<float>(v[1]),
                      static_cast<float>(v[2]), static_cast<float>(v[3])};
    h = *reinterpret_cast<const u4*>(&f);
    l = h;
  } else {
    bf8 hi, lo;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      __bf16 a, b;
      split_bf16(v[i], a, b);
      hi[i] = a;
      lo[i] = b;
    }
    h = *reinterpret_cast<const u4*>(&hi);
    l = *reinterpret_cast<const u4*>(&lo);
  }
}

// Panel P (depth K x width C, element (k, c) at P[k + c ld]) rounded into
// the packed format: depth slice s, column c, piece g (depth indices
// s BK + g VK ..) at 16-byte piece (s cp + c) 4 + g of each plane, planes
// kp cp elements apart; zero past K and C up to kp (a multiple of BK) and
// cp.  One thread per piece.
template <int PREC>
__global__ __launch_bounds__(256) void lowp_pack_kernel(const double* __restrict__ P, int64_t ld,
                                                        int64_t K, int64_t C, int64_t kp,
                                                        int64_t cp, u4* __restrict__ out) {
  constexpr int BK = Elem<PREC>::BK, VK = Elem<PREC>::VK;
  const int64_t pieces = kp / BK * cp * 4;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= pieces) return;
  const int64_t sc = idx >> 2, sl = sc / cp, c = sc - sl * cp;
  const int64_t k0 = sl * BK + (idx & 3) * VK;
  double v[VK];
#pragma unroll
  for (int i = 0; i < VK; ++i) v[i] = (c < C && k0 + i < K) ? P[k0 + i + c * ld] : 0.0;
  u4 h, l;
  round_piece<PREC>(v, h, l);
  out[idx] = h;
  if constexpr (PREC == 2) out[kp * cp / 8 + idx] = l;  // 8 bf16 per piece
}

// Accumulate the BM x BN tile over k in [kbeg, kend) (kbeg a multiple of
// BK).  NN (Y = X W): A is X, M x K with element (m, k) at X[m + k ldx]; B
// is the packed panel W.  TN (C = Q^T X): A is the packed panel Q; B is X,
// K x N with element (k, n) at X[k + n ldx].  pk: the packed panel's first
// plane, pl_off the pieces from it to the second (bf16x3 lo), cp its padded
// width.  vec: X allows 16-byte pair loads (TN only).
template <int PREC, class S, bool NN>
__device__ __forceinline__ void lowp_loop(const double* __restrict__ X, int64_t ldx,
                                          const u4* __restrict__ pk, int64_t pl_off,
                                          int64_t cp, int64_t m0,
                                          int64_t n0, int64_t M, int64_t N, int64_t kbeg,
                                          int64_t kend, bool vec, char* smem,
                                          f4 (&acc)[S::IB][S::JB]) {
  constexpr int BK = S::BK, SK = S::SK, NT = S::NT, VK = S::VK;
  constexpr int PL = Elem<PREC>::PLANES;
  constexpr int CS = NN ? S::BN : S::BM;       // panel columns of the tile
  constexpr int PC = CS * 4 / NT;              // panel pieces per thread and plane
  constexpr int GA = S::BM * BK / (VK * NT);   // NN: X rows (VK deep) per thread
  constexpr int PB = S::BN * BK / (2 * NT);    // TN: X pairs per thread
  static_assert(PC * NT == CS * 4, "whole panel pieces per thread");
  static_assert(!NN || GA * VK * NT == S::BM * BK, "whole X rows per thread");
  static_assert(NN || PB * 2 * NT == S::BN * BK, "whole X pairs per thread");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave % S::WGM) * S::WM, wn = (wave / S::WGM) * S::WN;
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  if (kbeg >= kend) return;

  const int64_t coff = NN ? n0 : m0;
  // depth slices in flight in registers: two (the loads of slice s + 2 are
  // issued while slice s + 1 waits to be stored), except for Y = X W in
  // f32 (one was faster: 1.56 against 1.61 ms per 20000 x 16000 x 256
  // sample) and in bf16x3 256 x 128 tiles (two rows of X per thread: two
  // sets do not fit in the registers)
  constexpr bool kTwoAhead = !(NN && (PREC == 1 || S::BM == 256));
  struct Regs {
    u4 pr[PL][PC];
    double xa[NN ? GA : 1][VK];
    double2 xb[NN ? 1 : PB];
  };
  Regs r0, r1;
  auto gload = [&](int64_t kc, Regs& R) __attribute__((always_inline)) {
    auto& pr = R.pr;
    auto& xa = R.xa;
    auto& xb = R.xb;
    // panel pieces: one contiguous block of CS * 4 pieces per plane
    const u4* blk = pk + ((kc / BK) * cp + coff) * 4;
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      pr[0][q] = blk[t + NT * q];
      if constexpr (PL == 2) pr[1][q] = blk[t + NT * q + pl_off];
    }
    if constexpr (NN) {
#pragma unroll
      for (int q = 0; q < GA; ++q) {
        const int e = t + NT * q;
        const int r = e % S::BM, g = e / S::BM;
        const int64_t gm = m0 + r, gk = kc + g * VK;
        const double* p = X + gm + gk * ldx;
#pragma unroll
        for (int i = 0; i < VK; ++i)
          xa[q][i] = (gm < M && gk + i < kend) ? p[i * ldx] : 0.0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int e = t + NT * q;
        const int kp = e % (BK / 2), c = e / (BK / 2);
        const int64_t gn = n0 + c, gk = kc + 2 * kp;
        xb[q] = ld_pair(X + gk + gn * ldx, gn < N && gk < kend, gn < N && gk + 1 < kend, vec);
      }
    }
  };

  auto sstore = [&](int stage, const Regs& R) __attribute__((always_inline)) {
    const auto& pr = R.pr;
    const auto& xa = R.xa;
    const auto& xb = R.xb;
    char* base = smem + stage * S::STAGE;
    // plane p of the A (rows BM) and B (rows BN) sides; 16-byte pieces
    // at row r, piece g: byte (r SK + g VK) * element size
    constexpr int ES = PREC == 1 ? 4 : 2;
    auto arow = [&](int p) { return base + p * S::BM * SK * ES; };
    auto brow = [&](int p) { return base + PL * S::BM * SK * ES + p * S::BN * SK * ES; };
    // panel pieces
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const int e = t + NT * q;
      const int c = e >> 2, g = e & 3;
#pragma unroll
      for (int p = 0; p < PL; ++p) {
        char* d = (NN ? brow(p) : arow(p)) + (c * SK + g * VK) * ES;
        *reinterpret_cast<u4*>(d) = pr[p][q];
      }
    }
    if constexpr (NN) {
#pragma unroll
      for (int q = 0; q < GA; ++q) {
        const int e = t + NT * q;
        const int r = e % S::BM, g = e / S::BM;
        u4 h, l;
        round_piece<PREC>(xa[q], h, l);
        *reinterpret_cast<u4*>(arow(0) + (r * SK + g * VK) * ES) = h;
        if constexpr (PL == 2) *reinterpret_cast<u4*>(arow(1) + (r * SK + g * VK) * ES) = l;
      }
    } else {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int e = t + NT * q;
        const int kp = e % (BK / 2), c = e / (BK / 2);
        if constexpr (PREC == 1) {
          float* Bs = reinterpret_cast<float*>(brow(0));
          *reinterpret_cast<fl2*>(Bs + c * SK + 2 * kp) =
              (fl2){static_cast<float>(xb[q].x), static_cast<float>(xb[q].y)};
        } else {
          __bf16 h0, l0, h1, l1;
          split_bf16(xb[q].x, h0, l0);
          split_bf16(xb[q].y, h1, l1);
          __bf16* Bh = reinterpret_cast<__bf16*>(brow(0));
          __bf16* Bl = reinterpret_cast<__bf16*>(brow(1));
          *reinterpret_cast<bf2*>(Bh + c * SK + 2 * kp) = (bf2){h0, h1};
          *reinterpret_cast<bf2*>(Bl + c * SK + 2 * kp) = (bf2){l0, l1};
        }
      }
    }
  };

  auto compute = [&](int stage) __attribute__((always_inline)) {
    if constexpr (PREC == 1) {
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
    } else {
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
    }
  };

  const int64_t ns = (kend - kbeg + BK - 1) / BK;
  if constexpr (!kTwoAhead) {
    gload(kbeg, r0);
    sstore(0, r0);
    __syncthreads();
    for (int64_t sl = 0; sl < ns; ++sl) {
      const int stage = static_cast<int>(sl & 1);
      if (sl + 1 < ns) gload(kbeg + (sl + 1) * BK, r0);
      compute(stage);
      if (sl + 1 < ns) sstore(stage ^ 1, r0);
      __syncthreads();
    }
    return;
  }
  // slice s: LDS stage s % 2, registers r0 (s even) or r1 (s odd)
  gload(kbeg, r0);
  if (ns > 1) gload(kbeg + BK, r1);
  sstore(0, r0);
  __syncthreads();
  auto step = [&](int64_t sl, int stage, Regs& next2, const Regs& next1)
                  __attribute__((always_inline)) {
    if (sl + 2 < ns) gload(kbeg + (sl + 2) * BK, next2);
    compute(stage);
    if (sl + 1 < ns) sstore(stage ^ 1, next1);
    __syncthreads();
  };
  for (int64_t sl = 0; sl < ns; sl += 2) {
    step(sl, 0, r0, r1);
    if (sl + 1 < ns) step(sl + 1, 1, r1, r0);
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

// Y = X W (X m-contiguous, W packed).  grid (M tiles, N tiles, split).
template <int PREC, class S>
__global__ __launch_bounds__(S::NT, 1) void lowp_nn_kernel(
    const double* __restrict__ X, int64_t ldx, const u4* __restrict__ Wp, int64_t pl_off,
    int64_t cp, double* __restrict__ Y, int64_t ldy, int64_t M, int64_t N, int64_t K,
    int64_t kchunk, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char smem[2 * S::STAGE];
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * S::BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * S::BN;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  f4 acc[S::IB][S::JB];
  lowp_loop<PREC, S, true>(X, ldx, Wp, pl_off, cp, m0, n0, M, N, kbeg, kend, false, smem, acc);
  store_tile<S>(acc, m0, n0, M, N, part, Y, ldy, 0);
}

// C = Q^T X (Q packed; X k-contiguous).  grid (N tiles, P tiles, split)
template <int PREC, class S>
__global__ __launch_bounds__(S::NT, 1) void lowp_tn_kernel(
    const u4* __restrict__ Qp, int64_t pl_off, int64_t cp, const double* __restrict__ X,
    int64_t ldx, double* __restrict__ C, int64_t ldc, int64_t P, int64_t N, int64_t K,
    int64_t kchunk, int transpose, int vec, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char smem[2 * S::STAGE];
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * S::BN;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * S::BM;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  f4 acc[S::IB][S::JB];
  lowp_loop<PREC, S, false>(X, ldx, Qp, pl_off, cp, m0, n0, P, N, kbeg, kend, vec != 0, smem,
                            acc);
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

// Layout of a low-precision product's scratch: the packed panel (planes of
// kp cp elements, kp the depth rounded up to 32, cp the panel width rounded
// up to the tile's panel side), then the split-K partials at a 256-byte
// boundary.  Both precisions take 4 bytes per packed element (one f32, or
// bf16 hi and lo).
struct LowpScratch {
  int64_t kp, cp, pack_doubles;
};
LowpScratch lowp_layout(int64_t K, int64_t panel_cols, int panel_side) {
  LowpScratch l;
  l.kp = round_up(K, 32);
  l.cp = round_up(panel_cols, panel_side);
  l.pack_doubles = round_up(l.kp * l.cp / 2, 32);
  return l;
}

template <int PREC>
int pack_panel(const double* P, int64_t ld, int64_t K, int64_t C, const LowpScratch& l,
               u4* out, hipStream_t s) {
  const int64_t pieces = l.kp / Elem<PREC>::BK * l.cp * 4;
  hipLaunchKernelGGL((lowp_pack_kernel<PREC>), dim3(static_cast<unsigned>(cdiv(pieces, 256))),
                     dim3(256), 0, s, P, ld, K, C, l.kp, l.cp, out);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

template <int PREC, class S>
int nn_impl(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y, int64_t ldy,
            int64_t M, int64_t N, int64_t K, int split, double* scratch, hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  if (K <= 0) return zero_matrix(Y, ldy, M, N, s);
  if (scratch == nullptr) return kEInval;
  const LowpScratch l = lowp_layout(K, N, S::BN);
  u4* pk = reinterpret_cast<u4*>(scratch);
  double* part = scratch + l.pack_doubles;
  const int64_t kc = split > 1 ? chunk_for(K, split, S::BK) : K;
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(M, S::BM)), static_cast<unsigned>(cdiv(N, S::BN)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmNNLowp, 2.0 * M * N * K * (PREC == 2 ? 3 : 1), 8.0 * (M * K + K * N + M * N), s);
    if (const int e = pack_panel<PREC>(W, ldw, K, N, l, pk, s)) return e;
    hipLaunchKernelGGL((lowp_nn_kernel<PREC, S>), grid, dim3(S::NT), 0, s, X, ldx, pk,
                       l.kp * l.cp / 8, l.cp, Y, ldy, M, N, K, kc,
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
            int64_t P, int64_t N, int64_t K, bool tr, int split, double* scratch, hipStream_t s) {
  if (P <= 0 || N <= 0) return kOk;
  if (K <= 0) return tr ? zero_matrix(C, ldc, N, P, s) : zero_matrix(C, ldc, P, N, s);
  if (scratch == nullptr) return kEInval;
  const LowpScratch l = lowp_layout(K, P, S::BM);
  u4* pk = reinterpret_cast<u4*>(scratch);
  double* part = scratch + l.pack_doubles;
  const int64_t kc = split > 1 ? chunk_for(K, split, S::BK) : K;
  const int nz = split > 1 ? static_cast<int>(cdiv(K, kc)) : 1;
  dim3 grid(static_cast<unsigned>(cdiv(N, S::BN)), static_cast<unsigned>(cdiv(P, S::BM)),
            static_cast<unsigned>(nz));
  {
    ProfScope ps(kKGemmTNLowp, 2.0 * P * N * K * (PREC == 2 ? 3 : 1), 8.0 * (K * P + K * N + P * N), s);
    if (const int e = pack_panel<PREC>(Qm, ldq, K, P, l, pk, s)) return e;
    hipLaunchKernelGGL((lowp_tn_kernel<PREC, S>), grid, dim3(S::NT), 0, s, pk, l.kp * l.cp / 8,
                       l.cp, X, ldx, C, ldc, P, N, K, kc, tr ? 1 : 0, pair_ok(X, ldx),
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

// panel side of the tile each product takes: Y = X W with panels up to 128
// wide takes 256 x 128 tiles (a 128 x 256 tile would multiply half a tile
// of zeros), C = Q^T X with panels Q up to 128 wide 128 x 256 tiles
bool nn_narrow(int64_t N) { return N <= TNS<1>::BN; }
bool tn_narrow(int64_t P) { return P <= NNS<1>::BM; }

}  // namespace

int lowp_split(int precision, bool nn, int64_t M, int64_t N, int64_t K) {
  // one eight-wave workgroup per CU in both precisions (bf16x3: two 61 KB
  // LDS stages; f32: about 145 VGPRs, so two waves per SIMD)
  (void)precision;
  const bool wide_tile = nn ? !nn_narrow(N) : tn_narrow(M);  // 128 x 256
  if (wide_tile) return choose_split_fill(M, N, K, 1, NNS<1>::BM, NNS<1>::BN);
  return choose_split_fill(M, N, K, 1, TNS<1>::BM, TNS<1>::BN);
}

size_t lowp_scratch_doubles(int precision, bool nn, int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  const int side = nn ? (nn_narrow(N) ? TNS<1>::BN : NNS<1>::BN)
                      : (tn_narrow(M) ? NNS<1>::BM : TNS<1>::BM);
  const LowpScratch l = lowp_layout(K, nn ? N : M, side);
  const int split = lowp_split(precision, nn, M, N, K);
  return static_cast<size_t>(l.pack_doubles) + partial_doubles(M, N, split) + 1;
}

int gemm_nn_lowp(int precision, const double* X, int64_t ldx, const double* W, int64_t ldw,
                 double* Y, int64_t ldy, int64_t M, int64_t N, int64_t K, int split,
                 double* scratch, hipStream_t s) {
  const bool narrow = nn_narrow(N);
  if (precision == 1)
    return narrow ? nn_impl<1, TNS<1>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, scratch, s)
                  : nn_impl<1, NNS<1>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, scratch, s);
  if (precision == 2)
    return narrow ? nn_impl<2, TNS<2>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, scratch, s)
                  : nn_impl<2, NNS<2>>(X, ldx, W, ldw, Y, ldy, M, N, K, split, scratch, s);
  return kEInval;
}

int gemm_tn_lowp(int precision, const double* Qm, int64_t ldq, const double* X, int64_t ldx,
                 double* C, int64_t ldc, int64_t P, int64_t N, int64_t K, bool transpose_out,
                 int split, double* scratch, hipStream_t s) {
  const bool narrow = tn_narrow(P);
  if (precision == 1)
    return narrow ? tn_impl<1, NNS<1>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, scratch, s)
                  : tn_impl<1, TNS<1>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, scratch, s);
  if (precision == 2)
    return narrow ? tn_impl<2, NNS<2>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, scratch, s)
                  : tn_impl<2, TNS<2>>(Qm, ldq, X, ldx, C, ldc, P, N, K, transpose_out, split, scratch, s);
  return kEInval;
}

}  // namespace qb
