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
// MFMA f64 16x16x4 lane layout (measured on gfx950):
//   A operand  lane l holds A[l % 16][l / 16]        (16 x 4)
//   B operand  lane l holds B[l / 16][l % 16]        (4 x 16)
//   result     lane l, element r holds D[l / 16 + 4 r][l % 16]
#include <cstdlib>

#include "qb_internal.hpp"

namespace qb {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BK = kTileK;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// BM x BN output tile per workgroup of WGM x WGN waves; each wave owns a
// (BM/WGM) x (BN/WGN) sub-tile.
template <int BM_, int BN_, int WGM_ = 2, int WGN_ = 2>
struct Shape {
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
  static constexpr int NT = 64 * WGM * WGN;          // threads per workgroup
  static constexpr int OCC = NT <= 256 ? 2 : 1;      // workgroups per CU (LDS bound)
  static constexpr int WM = BM / WGM, WN = BN / WGN; // wave sub-tile
  static constexpr int IB = WM / 16, JB = WN / 16;  // MFMA blocks per wave
  // LDS row strides (doubles).  MFMA fragment reads touch 16 rows x 4 depth
  // indices per instruction; with 32 eight-byte banks, a stride of BM + 16
  // (= 16 mod 32) puts the second group of 16 lanes on the other half of
  // the banks, and 18 (even) keeps the k-contiguous fragments conflict-free
  // while leaving every element pair 16-byte aligned for vector stores.
  static constexpr int SA_M = BM + 16;              // A stored [k][m] (m contiguous)
  static constexpr int SA_K = BK + 2;               // A stored [m][k] (k contiguous)
  static constexpr int SB_K = BK + 2;               // B stored [n][k] (k contiguous)
  static constexpr int A_LDS = (BK * SA_M > BM * SA_K) ? BK * SA_M : BM * SA_K;
  static constexpr int B_LDS = BN * SB_K;
  static constexpr int PA = (BM * BK) / NT, PB = (BN * BK) / NT;  // elements per thread per fill
};
// Big: two LDS stages of A and B take 73.7 KB, so two workgroups share a
// CU's 160 KB.  Small: a quarter of the work per workgroup, for outputs
// too small to give every CU a 128 x 128 tile.  Tall: 256 x 128 with 8
// waves (110 KB of LDS, one workgroup per CU) for products whose A operand
// is m-contiguous and tall: every depth slice reads 2 KB contiguous per
// column of A instead of 1 KB (a whole DRAM page instead of half of one),
// and the B slice is shared by twice the rows.
using Big = Shape<128, 128>;
using Small = Shape<64, 64>;
using Tall = Shape<256, 128, 4, 2>;
// Batched Gram matrices of panels w <= 16 or 32 wide: the tile matches the
// w x w output, so neither side of the MFMA work is padded to 64.  (Tiles
// narrow on one side only, 128 x 16 for R Omega or 16 x 128 for Q_i^T R,
// measured no faster than 64 x 64 there, and 256 x 64 for R Omega 60 %
// slower: those products are bound by the latency of their depth loops,
// and 64 x 64 tiles give the most workgroups.)
using BatchG16 = Shape<16, 16, 1, 1>;
using BatchG32 = Shape<32, 32, 2, 2>;
static_assert(Big::BM == kTileM && Big::BN == kTileN, "tile constants");

// A is "m-contiguous" when element (m, k) lies at X[m + k*ld] (column-major
// X); "k-contiguous" when it lies at X[k + m*ld] (the transposed operand Q^T).
// B is always k-contiguous: element (k, n) at B[k + n*ld].
template <class S, bool A_KCONTIG>
struct Tile {
  double ra[S::PA];
  double rb[S::PB];

  // 32-bit element offsets inside a tile (the launcher checks that 128 * ld
  // fits); the tile base pointer is uniform across the workgroup.
  __device__ __forceinline__ void load(const double* __restrict__ A, int64_t lda,
                                       const double* __restrict__ Bm, int64_t ldb, int64_t m0,
                                       int64_t n0, int64_t M, int64_t N, int64_t kc,
                                       int64_t kend) {
    const int t = threadIdx.x;
    const int64_t mlim = M - m0, nlim = N - n0, klim = kend - kc;
    const uint32_t la = static_cast<uint32_t>(lda), lb = static_cast<uint32_t>(ldb);
    const double* abase = A_KCONTIG ? A + kc + m0 * lda : A + m0 + kc * lda;
    const double* bbase = Bm + kc + n0 * ldb;
#pragma unroll
    for (int q = 0; q < S::PA; ++q) {
      const int e = t + S::NT * q;
      if (A_KCONTIG) {
        const int kk = e % BK, i = e / BK;
        ra[q] = (i < mlim && kk < klim)
                    ? abase[static_cast<uint32_t>(kk) + static_cast<uint32_t>(i) * la] : 0.0;
      } else {
        const int row = e % S::BM, col = e / S::BM;
        ra[q] = (row < mlim && col < klim)
                    ? abase[static_cast<uint32_t>(row) + static_cast<uint32_t>(col) * la] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < S::PB; ++q) {
      const int e = t + S::NT * q;
      const int kk = e % BK, nn = e / BK;
      rb[q] = (nn < nlim && kk < klim)
                  ? bbase[static_cast<uint32_t>(kk) + static_cast<uint32_t>(nn) * lb] : 0.0;
    }
  }

  __device__ __forceinline__ void store(double* As, double* Bs) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < S::PA; ++q) {
      const int e = t + S::NT * q;
      if (A_KCONTIG) As[(e / BK) * S::SA_K + (e % BK)] = ra[q];
      else As[(e / S::BM) * S::SA_M + (e % S::BM)] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < S::PB; ++q) {
      const int e = t + S::NT * q;
      Bs[(e / BK) * S::SB_K + (e % BK)] = rb[q];
    }
  }
};

// Interior tiles: 16-byte buffer loads.  The workgroup builds one buffer
// resource per operand at its tile origin; each lane keeps loop-invariant
// 32-bit byte offsets and the advance along k goes into the scalar offset,
// so a load costs no address arithmetic and no bounds test.  Used only when
// the whole tile, every depth slice, 16-byte alignment (base and even ld)
// and a byte extent below 2^31 are guaranteed (checked per workgroup).
typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufDword3 = 0x00020000;  // raw (untyped) buffer, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const double* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0,
                                           static_cast<int>(bytes), kBufDword3);
}

__device__ __forceinline__ double2 buf_load2(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                             uint32_t soff) {
  const i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(voff),
                                                        static_cast<int>(soff), 0);
  return __builtin_bit_cast(double2, v);
}

template <class S, bool A_KCONTIG>
struct FastTile {
  static constexpr int QA = S::PA / 2, QB = S::PB / 2;  // 16-byte loads per operand
  double2 ra[QA], rb[QB];
  uint32_t oa[QA], ob[QB];    // global byte offsets from the tile origin
  uint32_t la[QA], lb[QB];    // LDS element offsets

  __device__ __forceinline__ void setup(int64_t lda, int64_t ldb) {
    const int t = threadIdx.x;
    const uint32_t ua = static_cast<uint32_t>(lda), ub = static_cast<uint32_t>(ldb);
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e2 = t + S::NT * q;
      if (A_KCONTIG) {  // pairs along k: element (i, 2kp .. 2kp+1)
        const int kp = e2 % (BK / 2), i = e2 / (BK / 2);
        oa[q] = 8u * (2u * kp + static_cast<uint32_t>(i) * ua);
        la[q] = i * S::SA_K + 2 * kp;
      } else {          // pairs along m: element (2rp .. 2rp+1, col)
        const int rp = e2 % (S::BM / 2), col = e2 / (S::BM / 2);
        oa[q] = 8u * (2u * rp + static_cast<uint32_t>(col) * ua);
        la[q] = col * S::SA_M + 2 * rp;
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e2 = t + S::NT * q;
      const int kp = e2 % (BK / 2), nn = e2 / (BK / 2);
      ob[q] = 8u * (2u * kp + static_cast<uint32_t>(nn) * ub);
      lb[q] = nn * S::SB_K + 2 * kp;
    }
  }

  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rA, uint32_t sa,
                                       __amdgpu_buffer_rsrc_t rB, uint32_t sb) {
#pragma unroll
    for (int q = 0; q < QA; ++q) ra[q] = buf_load2(rA, oa[q], sa);
#pragma unroll
    for (int q = 0; q < QB; ++q) rb[q] = buf_load2(rB, ob[q], sb);
  }

  // every pair starts at an even LDS element (even strides, even offsets)
  __device__ __forceinline__ void store(double* As, double* Bs) const {
#pragma unroll
    for (int q = 0; q < QA; ++q) *reinterpret_cast<double2*>(As + la[q]) = ra[q];
#pragma unroll
    for (int q = 0; q < QB; ++q) *reinterpret_cast<double2*>(Bs + lb[q]) = rb[q];
  }
};

// MFMA row permutation: the A operand of lane l carries tile row
// perm(l % 16), perm(rho) = 4 (rho % 4) + rho / 4.  With the result layout
// D[l/16 + 4r][l%16] this puts rows 4 (l / 16) + r, r = 0..3, in the four
// result elements of lane l: every lane holds four consecutive rows of one
// column, so epilogues move them with 16-byte accesses.
__device__ __forceinline__ int perm16(int rho) { return 4 * (rho & 3) + (rho >> 2); }

// MFMA work of one depth slice held in LDS
template <class S, bool A_KCONTIG>
__device__ __forceinline__ void mma_slice(const double* Ac, const double* Bc,
                                          d4 (&acc)[S::IB][S::JB]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave % S::WGM) * S::WM, wn = (wave / S::WGM) * S::WN;
  const int lr = lane & 15, lk = lane >> 4;
  const int pr = perm16(lr);
#pragma unroll
  for (int k4 = 0; k4 < BK / 4; ++k4) {
    double a[S::IB], b[S::JB];
    const int kq = 4 * k4 + lk;
#pragma unroll
    for (int i = 0; i < S::IB; ++i) {
      const int mrow = wm + 16 * i + pr;
      a[i] = A_KCONTIG ? Ac[mrow * S::SA_K + kq] : Ac[kq * S::SA_M + mrow];
    }
#pragma unroll
    for (int j = 0; j < S::JB; ++j) b[j] = Bc[(wn + 16 * j + lr) * S::SB_K + kq];
#pragma unroll
    for (int i = 0; i < S::IB; ++i)
#pragma unroll
      for (int j = 0; j < S::JB; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// Accumulate the workgroup tile over k in [kbeg, kend).  As/Bs hold two
// LDS stages each: slice s + 1 is written to the free stage and slice s + 2
// is in flight in registers while slice s is multiplied.
template <class S, bool A_KCONTIG>
__device__ __forceinline__ void mma_loop(const double* __restrict__ A, int64_t lda,
                                         const double* __restrict__ Bm, int64_t ldb, int64_t m0,
                                         int64_t n0, int64_t M, int64_t N, int64_t kbeg,
                                         int64_t kend, bool vec, double* As, double* Bs,
                                         d4 (&acc)[S::IB][S::JB]) {
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
  if (kbeg >= kend) return;

  const int64_t klen = kend - kbeg;
  const int64_t ext_a = A_KCONTIG ? klen + (S::BM - 1) * lda : S::BM + (klen - 1) * lda;
  const int64_t ext_b = klen + (S::BN - 1) * ldb;
  const bool fast = vec && m0 + S::BM <= M && n0 + S::BN <= N && klen % BK == 0 &&
                    8 * ext_a < (int64_t(1) << 31) && 8 * ext_b < (int64_t(1) << 31);
  if (fast) {
    const double* a0 = A_KCONTIG ? A + kbeg + m0 * lda : A + m0 + kbeg * lda;
    const double* b0 = Bm + kbeg + n0 * ldb;
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(a0, 8 * ext_a);
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(b0, 8 * ext_b);
    // byte advance of one depth slice
    const uint32_t da = static_cast<uint32_t>(8 * (A_KCONTIG ? BK : BK * lda));
    const uint32_t db = static_cast<uint32_t>(8 * BK);
    const int nslice = static_cast<int>(klen / BK);
    FastTile<S, A_KCONTIG> tl;
    tl.setup(lda, ldb);
    tl.load(rA, 0u, rB, 0u);
    tl.store(As, Bs);
    if (nslice > 1) tl.load(rA, da, rB, db);
    lds_barrier();
    int stage = 0;
    for (int sl = 0; sl < nslice; ++sl) {
      if (sl + 1 < nslice) {
        tl.store(As + (stage ^ 1) * S::A_LDS, Bs + (stage ^ 1) * S::B_LDS);
        if (sl + 2 < nslice) tl.load(rA, (sl + 2) * da, rB, (sl + 2) * db);
      }
      mma_slice<S, A_KCONTIG>(As + stage * S::A_LDS, Bs + stage * S::B_LDS, acc);
      lds_barrier();
      stage ^= 1;
    }
    return;
  }

  Tile<S, A_KCONTIG> tl;
  tl.load(A, lda, Bm, ldb, m0, n0, M, N, kbeg, kend);
  tl.store(As, Bs);
  if (kbeg + BK < kend) tl.load(A, lda, Bm, ldb, m0, n0, M, N, kbeg + BK, kend);
  lds_barrier();
  int stage = 0;
  for (int64_t kc = kbeg; kc < kend; kc += BK) {
    if (kc + BK < kend) {
      tl.store(As + (stage ^ 1) * S::A_LDS, Bs + (stage ^ 1) * S::B_LDS);
      if (kc + 2 * BK < kend) tl.load(A, lda, Bm, ldb, m0, n0, M, N, kc + 2 * BK, kend);
    }
    mma_slice<S, A_KCONTIG>(As + stage * S::A_LDS, Bs + stage * S::B_LDS, acc);
    lds_barrier();
    stage ^= 1;
  }
}

// first of the four consecutive tile rows held by this lane for block i,
// and the tile column for block j
template <class S>
__device__ __forceinline__ int acc_row0(int i) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave % S::WGM) * S::WM + 16 * i + 4 * (lane >> 4);
}
template <class S>
__device__ __forceinline__ int acc_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave / S::WGM) * S::WN + 16 * j + (lane & 15);
}

__device__ __forceinline__ bool vec_ok_dev(const double* p, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && (ld & 1) == 0;
}

// four consecutive rows [row0, row0 + 4) of column col of X (ld); vec: X and
// ld allow 16-byte accesses at even rows
__device__ __forceinline__ d4 load4(const double* __restrict__ X, int64_t ld, int64_t row0,
                                    int64_t col, int64_t M, int64_t N, bool vec) {
  d4 v = (d4){0.0, 0.0, 0.0, 0.0};
  if (col >= N) return v;
  const double* p = X + row0 + col * ld;
  if (vec && row0 + 3 < M) {
    const double2 lo = *reinterpret_cast<const double2*>(p);
    const double2 hi = *reinterpret_cast<const double2*>(p + 2);
    v = (d4){lo.x, lo.y, hi.x, hi.y};
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (row0 + r < M) v[r] = p[r];
  }
  return v;
}
__device__ __forceinline__ void store4(double* __restrict__ X, int64_t ld, int64_t row0,
                                       int64_t col, int64_t M, int64_t N, bool vec, d4 v) {
  if (col >= N) return;
  double* p = X + row0 + col * ld;
  if (vec && row0 + 3 < M) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (row0 + r < M) p[r] = v[r];
  }
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

// out(M x N) = alpha * sum_s part[s] + beta * out; part[s] has ld ldp;
// transposed store puts element (i, j) at out[j + i*ldo].  Optional
// per-block sums of squares of the result.
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int split,
                                                     int64_t ldp, double* __restrict__ out,
                                                     int64_t ldo, int64_t M, int64_t N,
                                                     double alpha, double beta, int transpose_out,
                                                     double* __restrict__ sq_part) {
  __shared__ double red[4];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = M * N;
  double sq = 0.0;
  if (idx < total) {
    const int64_t i = idx % M, j = idx / M;
    const int64_t pidx = i + j * ldp, pstride = ldp * N;
    double s = 0.0;
    for (int z = 0; z < split; ++z) s += part[z * pstride + pidx];
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
                   hipStream_t s) {
  const int64_t total = M * N;
  if (sq_part == nullptr && nz >= 2 * kWideG && total <= (int64_t(1) << 18)) {
    constexpr int OPB = 256 / kWideG;
    *nb = static_cast<unsigned>(cdiv(total, OPB));
    hipLaunchKernelGGL(reduce_wide_kernel<kWideG>, dim3(*nb), dim3(256), 0, s, part, nz, ldp, out,
                       ldo, M, N, alpha, beta, tr ? 1 : 0);
    return;
  }
  *nb = static_cast<unsigned>(cdiv(total, 256));
  hipLaunchKernelGGL(reduce_kernel, dim3(*nb), dim3(256), 0, s, part, nz, ldp, out, ldo, M, N,
                     alpha, beta, tr ? 1 : 0, sq_part);
}

// R -= Q B; per-workgroup sum of squares of the updated tile.
// grid: (M tiles, N tiles)
template <class S>
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
  const int64_t m0 = static_cast<int64_t>(blockIdx.x) * S::BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.y) * S::BN;
  d4 acc[S::IB][S::JB];
  mma_loop<S, false>(Qm, ldq, B, ldb, m0, n0, M, N, 0, K, vec_ab != 0, As, Bs, acc);
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < S::IB; ++i) {
    const int64_t row0 = m0 + acc_row0<S>(i);
    d4 rv[S::JB];
#pragma unroll
    for (int j = 0; j < S::JB; ++j) rv[j] = load4(R, ldr, row0, n0 + acc_col<S>(j), M, N, vec_r);
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t col = n0 + acc_col<S>(j);
      const d4 v = rv[j] - acc[i][j];
      store4(R, ldr, row0, col, M, N, vec_r, v);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < M && col < N) sq += v[r] * v[r];
    }
  }
  const double tot = block_sum(sq, red);
  if (threadIdx.x == 0) sq_part[blockIdx.x + static_cast<int64_t>(blockIdx.y) * gridDim.x] = tot;
}

// ---- batched products ------------------------------------------------------
// Workgroup -> (problem, tile) by binary search over the problems' first
// workgroup indices; then the same tile loop and epilogues as above.
template <class S, int OP>
__global__ __launch_bounds__(S::NT, S::OCC) void gemm_batched_kernel(
    const BatchGemm* __restrict__ desc, int count) {
  __shared__ __attribute__((aligned(16))) double As[2 * S::A_LDS];
  __shared__ __attribute__((aligned(16))) double Bs[2 * S::B_LDS];
  __shared__ double red[S::NT / 64];
  const int64_t blk = blockIdx.x;
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
  // the old C of a downdate (or of an NN product with beta) is read before
  // the MMA loop, so its latency overlaps the operand loads
  const bool vc = vec_ok_dev(g.C, g.ldc);
  const bool need = g.ksplit == 1 && ((OP == kBatchDD) || (OP == kBatchNN && g.beta != 0.0));
  d4 old[S::IB][S::JB];
#pragma unroll
  for (int i = 0; i < S::IB; ++i)
#pragma unroll
    for (int j = 0; j < S::JB; ++j)
      old[i][j] = need ? load4(g.C, g.ldc, m0 + acc_row0<S>(i), n0 + acc_col<S>(j), M, N, vc)
                       : (d4){0.0, 0.0, 0.0, 0.0};
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
#pragma unroll
    for (int j = 0; j < S::JB; ++j) {
      const int64_t col = n0 + acc_col<S>(j);
      d4 v;
      if (OP == kBatchNN) v = g.alpha * acc[i][j] + g.beta * old[i][j];
      else if (OP == kBatchTN) v = acc[i][j];
      else v = old[i][j] - acc[i][j];
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

// C from the depth chunks of the problems with ksplit > 1, in chunk order;
// kBatchRed elements of C per workgroup
template <int OP>
__global__ __launch_bounds__(256) void gemm_batched_reduce_kernel(
    const BatchGemm* __restrict__ desc, int count) {
  __shared__ double red[4];
  const int64_t blk = blockIdx.x;
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

}  // namespace

int choose_split(int64_t M, int64_t N, int64_t K, int slots_per_cu) {
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
  return static_cast<int>(s);
}

size_t partial_doubles(int64_t M, int64_t N, int split) {
  return split > 1 ? static_cast<size_t>(part_ld(M)) * N * split : 0;
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
  // unsplit products with too few 128 x 128 tiles to fill the chip (the
  // T^{-1} application, short projections) take 64 x 64 tiles; tall
  // products with enough 256-row tiles for one workgroup per CU take Tall
  const bool small = nz == 1 && cdiv(M, Big::BM) * cdiv(N, Big::BN) < kNumCU;
  const bool tall = !small && use_tall(M, N, nz);
  {
    ProfScope ps(small ? kKGemmNNSmall : tall ? kKGemmNNTall : kKGemmNN, 2.0 * M * N * K,
                 8.0 * (M * K + K * N + M * N * (beta != 0.0 ? 2 : 1)), s);
    double* pp = nz > 1 ? part : nullptr;
    if (small)
      launch_nn<Small>(X, ldx, W, ldw, Y, ldy, M, N, K, kc, nz, alpha, beta, pp, ldp, s);
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
    launch_reduce(part, nz, ldp, Y, ldy, M, N, alpha, beta, false, nullptr, &nb, s);
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
  dim3 grid;
  {
    ProfScope ps(small ? kKGemmTNSmall : kKGemmTN, 2.0 * P * N * K, 8.0 * (K * P + K * N + P * N), s);
    double* pp = nz > 1 ? part : nullptr;
    double* sqp = nz > 1 ? static_cast<double*>(nullptr) : sq_part;
    grid = small ? launch_tn<Small>(Qm, ldq, X, ldx, C, ldc, P, N, K, kc, nz, transpose_out, pp,
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

size_t downdate_partials(int64_t M, int64_t N) {
  return static_cast<size_t>(cdiv(M, Big::BM)) * static_cast<size_t>(cdiv(N, Big::BN));
}

int downdate(double* R, int64_t ldr, const double* Qm, int64_t ldq, const double* B, int64_t ldb,
             int64_t M, int64_t N, int64_t K, double* sq_part, int* sq_count, hipStream_t s) {
  if (M <= 0 || N <= 0) { if (sq_count) *sq_count = 0; return kOk; }
  if (!ld_fits(ldq) || !ld_fits(ldb)) return kEInval;
  // 128 x 128 tiles, two workgroups per CU: the read-modify-write of R in
  // one workgroup's epilogue overlaps the other's MFMA work (measured: the
  // 256-row tile with one workgroup per CU is 16 % slower here)
  const dim3 grid(static_cast<unsigned>(cdiv(M, Big::BM)), static_cast<unsigned>(cdiv(N, Big::BN)));
  {
    ProfScope ps(kKDowndate, 2.0 * M * N * K, 8.0 * (2 * M * N + M * K + K * N), s);
    hipLaunchKernelGGL(downdate_kernel<Big>, grid, dim3(Big::NT), 0, s, R, ldr, Qm, ldq, B, ldb,
                       M, N, K, sq_part, vec_ok(R, ldr), vec_ok(Qm, ldq) & vec_ok(B, ldb));
  }
  QB_HIP_TRY(hipGetLastError());
  if (sq_count) *sq_count = static_cast<int>(grid.x * grid.y);
  return kOk;
}

namespace {
template <class S>
void launch_batched(int op, const BatchGemm* desc, int count, int64_t total_tiles, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(total_tiles));
  if (op == kBatchNN)
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchNN>), grid, dim3(S::NT), 0, s, desc, count);
  else if (op == kBatchTN)
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchTN>), grid, dim3(S::NT), 0, s, desc, count);
  else
    hipLaunchKernelGGL((gemm_batched_kernel<S, kBatchDD>), grid, dim3(S::NT), 0, s, desc, count);
}
}  // namespace

void batch_tile_dims(int cls, int* bm, int* bn) {
  switch (cls) {
    case kTileG16: *bm = BatchG16::BM; *bn = BatchG16::BN; return;
    case kTileG32: *bm = BatchG32::BM; *bn = BatchG32::BN; return;
    default: *bm = Small::BM; *bn = Small::BN; return;
  }
}

int gemm_batched(int op, int cls, const BatchGemm* desc, int count, int64_t total_tiles,
                 int prof_id, double flops, hipStream_t s) {
  if (count <= 0 || total_tiles <= 0) return kOk;
  if (op == kBatchDD && cls != kTile64) return kEInval;
  ProfScope ps(prof_id, flops, 0.0, s);
  switch (cls) {
    case kTileG16: launch_batched<BatchG16>(op, desc, count, total_tiles, s); break;
    case kTileG32: launch_batched<BatchG32>(op, desc, count, total_tiles, s); break;
    default: launch_batched<Small>(op, desc, count, total_tiles, s); break;
  }
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int gemm_batched_reduce(int op, const BatchGemm* desc, int count, int64_t total_rblocks,
                        int prof_id, hipStream_t s) {
  if (count <= 0 || total_rblocks <= 0) return kOk;
  if (op == kBatchDD) return kEInval;
  const dim3 grid(static_cast<unsigned>(total_rblocks));
  ProfScope ps(prof_id, 0.0, 0.0, s);
  if (op == kBatchNN)
    hipLaunchKernelGGL(gemm_batched_reduce_kernel<kBatchNN>, grid, dim3(256), 0, s, desc, count);
  else
    hipLaunchKernelGGL(gemm_batched_reduce_kernel<kBatchTN>, grid, dim3(256), 0, s, desc, count);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

}  // namespace qb
