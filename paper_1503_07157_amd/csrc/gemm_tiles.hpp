// Tile machinery of the FP64 MFMA GEMM kernels (gfx950), shared by the
// single-matrix products (k_gemm64.hip) and the batched ones
// (k_gemm_batched.hip): tile shapes, operand staging through LDS (guarded
// and buffer-load paths), the MFMA slice and depth loop, epilogue helpers.
//
// MFMA f64 16x16x4 lane layout (measured on gfx950):
//   A operand  lane l holds A[l % 16][l / 16]        (16 x 4)
//   B operand  lane l holds B[l / 16][l % 16]        (4 x 16)
//   result     lane l, element r holds D[l / 16 + 4 r][l % 16]
#pragma once

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
// every depth slice, 16-byte alignment (base and even ld) and a byte extent
// below 2^31 are guaranteed, and the tile is whole or its missing rows or
// columns read as zero (checked per workgroup in mma_loop).
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
  // Q^T X products (A k-contiguous): LLVM's interleaving of LDS reads with
  // the MFMA chain (iglp_opt(1)) cut gemm_tn from 259 to 249 ms per
  // 20000 x 16000 factorisation; on the other products it was neutral or
  // slower (the downdate 196 -> 203 ms), and iglp_opt(0) slower everywhere
  if constexpr (A_KCONTIG) __builtin_amdgcn_iglp_opt(1);
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
  // The buffer-load path covers the whole slices of the depth range; a
  // ragged last slice (fewer than BK) follows on the guarded path below.
  // A k-contiguous operand tile that runs past the last valid row or column
  // (a partial edge tile, or a panel narrower than the tile) still takes the
  // buffer-load path: with ld >= the depth, every element of a row or column
  // beyond the valid ones lies at or past the resource's extent, where
  // buffer loads return zero.  An m-contiguous A tile must be whole.  The
  // lane offsets of the whole tile stay below 2^31 bytes (no 32-bit wrap
  // back into the valid range); the resources cover the valid part.
  const int64_t kfast = klen - klen % BK;
  const int64_t mv = M - m0 < S::BM ? M - m0 : S::BM;
  const int64_t nv = N - n0 < S::BN ? N - n0 : S::BN;
  const int64_t full_a = A_KCONTIG ? kfast + (S::BM - 1) * lda : S::BM + (kfast - 1) * lda;
  const int64_t full_b = kfast + (S::BN - 1) * ldb;
  const int64_t ext_a = A_KCONTIG ? kfast + (mv - 1) * lda : full_a;
  const int64_t ext_b = kfast + (nv - 1) * ldb;
  const bool fast = vec && kfast > 0 && (A_KCONTIG ? lda >= kfast : m0 + S::BM <= M) &&
                    ldb >= kfast && 8 * full_a < (int64_t(1) << 31) &&
                    8 * full_b < (int64_t(1) << 31);
  if (fast) {
    const double* a0 = A_KCONTIG ? A + kbeg + m0 * lda : A + m0 + kbeg * lda;
    const double* b0 = Bm + kbeg + n0 * ldb;
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(a0, 8 * ext_a);
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(b0, 8 * ext_b);
    // byte advance of one depth slice
    const uint32_t da = static_cast<uint32_t>(8 * (A_KCONTIG ? BK : BK * lda));
    const uint32_t db = static_cast<uint32_t>(8 * BK);
    const int nslice = static_cast<int>(kfast / BK);
    FastTile<S, A_KCONTIG> tl;
    tl.setup(lda, ldb);
    tl.load(rA, 0u, rB, 0u);
    tl.store(As, Bs);
    if (nslice > 1) tl.load(rA, da, rB, db);
    lds_barrier();
    int stage = 0;
    int sl = 0;
    // Steady state as one basic block (no per-slice branches) for the
    // Q^T X products with tiles of 128 or 256 rows and the 128 x 128 tiles;
    // for the 128 x 128 tiles of Y = X W and the downdate the next slice's
    // LDS stores and global loads are dealt between the MFMAs, and the LDS
    // operand reads one per MFMA (sched_group_barrier).  Measured per
    // 20000 x 16000 factorisation: downdate 196 -> 191 ms, gemm_tn 249 ->
    // 244 ms; the 256 x 128 tiles of Y = X W keep the plain loop (peeled,
    // 248 -> 258 ms), and so do the 64 x 64 tiles (the Gram matrices,
    // peeled 19 -> 21 ms).
    constexpr bool kPeel = S::BM >= 128 && (A_KCONTIG || S::BM == 128);
    if constexpr (kPeel) {
      for (; sl + 2 < nslice; ++sl) {
        tl.store(As + (stage ^ 1) * S::A_LDS, Bs + (stage ^ 1) * S::B_LDS);
        tl.load(rA, (sl + 2) * da, rB, (sl + 2) * db);
        mma_slice<S, A_KCONTIG>(As + stage * S::A_LDS, Bs + stage * S::B_LDS, acc);
        if constexpr (!A_KCONTIG && S::BM == 128) {
          constexpr int kMem = FastTile<S, A_KCONTIG>::QA + FastTile<S, A_KCONTIG>::QB;
          constexpr int kMfma = (BK / 4) * S::IB * S::JB;
          constexpr int kReads = (BK / 4) * (S::IB + S::JB);
          static_assert(4 * kMem + kReads == kMfma, "one MFMA per LDS read after the stores");
#pragma unroll
          for (int g = 0; g < kMem; ++g) {
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // global (buffer) load
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          }
#pragma unroll
          for (int g = 0; g < kReads; ++g) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          }
        }
        lds_barrier();
        stage ^= 1;
      }
    }
    for (; sl < nslice; ++sl) {
      if (sl + 1 < nslice) {
        tl.store(As + (stage ^ 1) * S::A_LDS, Bs + (stage ^ 1) * S::B_LDS);
        if (sl + 2 < nslice) tl.load(rA, (sl + 2) * da, rB, (sl + 2) * db);
      }
      mma_slice<S, A_KCONTIG>(As + stage * S::A_LDS, Bs + stage * S::B_LDS, acc);
      lds_barrier();
      stage ^= 1;
    }
    if (kfast == klen) return;
    // ragged last slice: one guarded load into a free stage (every wave
    // has passed the barrier after the last multiply)
    Tile<S, A_KCONTIG> tt;
    tt.load(A, lda, Bm, ldb, m0, n0, M, N, kbeg + kfast, kend);
    tt.store(As, Bs);
    lds_barrier();
    mma_slice<S, A_KCONTIG>(As, Bs, acc);
    lds_barrier();
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

}  // namespace
}  // namespace qb
