// orth(X) (Section 2.4) as Cholesky QR applied twice, with column dropping.
//
// One pass: G = X^T X (split-K MFMA product), upper Cholesky G = T^T T in
// natural column order where column c is dropped when its pivot
//     d_c = G_cc - sum_{l kept, l < c} T_lc^2  <=  2^-40 * max_j G_jj,
// then Q = X_kept T^{-1}.  The paper assumes full-rank blocks (Proposition
// 3.1); dropping handles blocks that are numerically rank deficient.  The
// kept columns of Q come first, in their original order, followed by zero
// columns, and the kept count is left on the device.
//
// Cholesky, panels up to 128 wide: one workgroup, G in LDS (scaled by an
// exact power of two), right-looking and blocked by 16 columns.  One wave
// factors a 16-column panel in registers, exchanging values across lanes
// with readlane (no barrier inside the panel), with the next pivot's
// reciprocal square root computed while the current column's updates
// issue; the trailing update G22 -= L21 L21^T runs on
// v_mfma_f64_16x16x4_f64 over the other waves while wave 0 factors the
// next panel (look-ahead).  Wider panels (129..256) are blocked 128 +
// (w - 128): the LDS factorisation of the leading block, the Schur
// complement of the trailing block by two small MFMA products, the LDS
// factorisation of that, and the off-diagonal block of the inverse by two
// more products (chol_inv_wide), all with the scale and drop threshold of
// the whole Gram matrix.
//
// Inverse: T^{-1} of the kept part, blocked in LDS (16 x 16 diagonal blocks
// by substitution, joined pairwise with MFMA products) for blocks up to 128.
#include <algorithm>
#include <utility>

#include "qb_internal.hpp"

namespace qb {
namespace {

constexpr double kDropRel = 0x1p-40;

// compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// value of v in lane l (l uniform)
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u)), l));
  const unsigned hi = static_cast<unsigned>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u >> 32)), l));
  return __longlong_as_double(
      static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

constexpr int kPanel = 16;  // Cholesky panel width

// Factor panel columns [p, p + 16) of the LDS matrix (Ts[j * TS + i] holds
// L[i][j], i >= j; rows p.. hold the updated trailing part).  Run by one
// wave: lane l holds rows p + l + 64 a.  Column c is kept when its pivot
// exceeds thresh; a dropped column becomes zero.  Sets flag[c] and
// rdiag[c] = 1 / L[c][c] (1 for a dropped or padding column).  G was scaled
// so that every pivot above thresh lies in (2^-41, 2).
//
// The column loop needs no per-lane tests: scaling a whole column by
// 1/sqrt(d) leaves sqrt(d) on the diagonal lane, and lanes above the
// diagonal only carry values nobody reads (cleared when written back).
//
// Column chain.  With G' the matrix after the updates of the columns before
// c, L[c+1][c] = G'[c+1][c] r_c and the next pivot is
// d_{c+1} = G'[c+1][c+1] - L[c+1][c]^2: one product and one fma of broadcast
// values, the same operations, in the same order, as the vector update of
// column c+1 performs on lane c+1.  So r_{c+1} = 1/sqrt(d_{c+1}) is formed
// while the vector updates of column c are issued, one stage between two
// updates, and the wave's in-order issue hides the chain's latency.
// 1/sqrt: the hardware estimate y (relative error below 2^-24) with one
// third-order correction y + y e (1/2 + 3/8 e), e = 1 - d y^2, to about
// one ulp.
//
// RA row slots per lane are live (rows p .. p + 64 RA - 1 cover the rows
// left).  Rows past WMAX are read from and written to the padding row
// (index WMAX) of each LDS column, which nothing else reads, so the loads
// and stores need no masks.
template <int WMAX, int RA>
__device__ __forceinline__ void chol_panel(double* Ts, int p, int w, double thresh, bool gpos,
                                           int* flag, double* rdiag) {
  constexpr int TS = WMAX + 1;
  constexpr int kStages = 7;
  // opaque per call, so per-lane values are not hoisted out of the panel loop
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  double x[RA][kPanel];
  static_for<kPanel>([&](auto jj) {
    static_for<RA>([&](auto a) {
      const int i = p + lane + 64 * a;
      const double v = Ts[(p + jj) * TS + (i < WMAX ? i : WMAX)];
      x[a][jj] = (i < WMAX) ? v : 0.0;
    });
  });
  // lane J collects flag and 1 / L[c][c] of column c = p + J, written once
  // after the panel so that no lane-0 store sits in the column chain
  int fl = 0;
  double rd = 1.0;
  // the first pivot and its reciprocal square root, unhidden
  double r;
  bool keep;
  {
    const double d = readlane_d(x[0][0], 0);
    const double y = __builtin_amdgcn_rsq(d);
    const double e = fma(-(d * y), y, 1.0);
    const double yc = fma(y * e, fma(0.375, e, 0.5), y);
    keep = (p < w) && gpos && (d > thresh);
    r = keep ? yc : 0.0;
  }
  static_for<kPanel>([&](auto jj) {
    constexpr int J = decltype(jj)::value;
    // chain state for column J + 1 (its broadcast inputs read before this
    // column's scaling and updates)
    double g10 = 0.0, g11 = 0.0, t = 0.0, dn = 0.0, y = 0.0, u = 0.0, e = 0.0, q = 0.0, pc = 0.0;
    if constexpr (J + 1 < kPanel) {
      g10 = readlane_d(x[0][J], J + 1);
      g11 = readlane_d(x[0][J + 1], J + 1);
    }
    auto stage = [&](auto sidx) {
      constexpr int S = decltype(sidx)::value;
      if constexpr (J + 1 < kPanel) {
        if constexpr (S == 0) { t = g10 * r; asm volatile("" : "+v"(t)); }
        if constexpr (S == 1) { dn = fma(-t, t, g11); asm volatile("" : "+v"(dn)); }
        if constexpr (S == 2) { y = __builtin_amdgcn_rsq(dn); asm volatile("" : "+v"(y)); }
        if constexpr (S == 3) { u = dn * y; asm volatile("" : "+v"(u)); }
        if constexpr (S == 4) { e = fma(-u, y, 1.0); asm volatile("" : "+v"(e)); }
        if constexpr (S == 5) {
          q = y * e;
          pc = fma(0.375, e, 0.5);
          asm volatile("" : "+v"(q), "+v"(pc));
        }
        if constexpr (S == 6) { y = fma(q, pc, y); asm volatile("" : "+v"(y)); }
      }
    };
    static_for<RA>([&](auto a) { x[a][J] *= r; });
    stage(std::integral_constant<int, 0>{});
    // rank-one update of the panel's later columns, one chain stage after
    // each; the multiplier of column c + 1 is the chain's t = L[c+1][c]
    static_for<kPanel - 1 - J>([&](auto tt) {
      constexpr int T = decltype(tt)::value;
      constexpr int K = J + 1 + T;
      double lk;  // L[p + K][c]
      if constexpr (T == 0) lk = t;
      else lk = readlane_d(x[0][J], K);
      static_for<RA>([&](auto a) {
        x[a][K] = fma(-x[a][J], lk, x[a][K]);
        // keep the update here; left to itself the compiler sinks it to the
        // use of column K and holds every broadcast value in scalar registers
        asm volatile("" : "+v"(x[a][K]));
      });
      if constexpr (T + 1 < kStages) stage(std::integral_constant<int, T + 1>{});
    });
    // stages left over when fewer updates than stages remain
    static_for<kStages>([&](auto sidx) {
      constexpr int S = decltype(sidx)::value;
      if constexpr (S >= 1 && S >= kPanel - J) stage(sidx);
    });
    fl = (lane == J) ? (keep ? 1 : 0) : fl;
    rd = (lane == J) ? (keep ? r : 1.0) : rd;
    if constexpr (J + 1 < kPanel) {
      keep = (p + J + 1 < w) && gpos && (dn > thresh);
      r = keep ? y : 0.0;
    }
  });
  if (lane < kPanel) {
    flag[p + lane] = fl;
    rdiag[p + lane] = rd;
  }
  static_for<kPanel>([&](auto jj) {
    static_for<RA>([&](auto a) {
      const int i = p + lane + 64 * a;
      Ts[(p + jj) * TS + (i < WMAX ? i : WMAX)] = (a > 0 || lane >= jj) ? x[a][jj] : 0.0;
    });
  });
}

// Trailing update after panel p: L[i][j] -= sum_t L[i][p + t] L[j][p + t]
// for p + 16 <= j <= i < 16 ceil(w / 16), as 16 x 16 MFMA blocks (diagonal
// blocks are updated whole; their upper halves are cleared when their own
// panel is written).  Block (bi, bj), bj <= bi, counts from q = p + 16.
__device__ __forceinline__ void chol_trail_block(double* Ts, int TS, int p, int bi, int bj) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int q = p + kPanel;
  const int lr = lane & 15, lk = lane >> 4;
  double a[4], b[4];
#pragma unroll
  for (int k4 = 0; k4 < 4; ++k4) {
    a[k4] = Ts[(p + 4 * k4 + lk) * TS + q + 16 * bi + lr];
    b[k4] = Ts[(p + 4 * k4 + lk) * TS + q + 16 * bj + lr];
  }
  d4 acc = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k4 = 0; k4 < 4; ++k4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k4], b[k4], acc, 0, 0, 0);
  double* col = Ts + (q + 16 * bj + lr) * TS + q + 16 * bi + lk;
#pragma unroll
  for (int r = 0; r < 4; ++r) col[4 * r] -= acc[r];
}

// (bi, bj) of lower-triangle index job = bi (bi + 1) / 2 + bj, bj <= bi
__device__ __forceinline__ void tri_index(int job, int& bi, int& bj) {
  bi = static_cast<int>((sqrtf(8.0f * job + 1.0f) - 1.0f) * 0.5f);
  while ((bi + 1) * (bi + 2) / 2 <= job) ++bi;
  while (bi * (bi + 1) / 2 > job) --bi;
  bj = job - bi * (bi + 1) / 2;
}

// Source of a Gram matrix (or of its whole-matrix counterpart Gd): G with
// leading dimension ld, or, when part is set, the sum of the nz depth-chunk
// partial products part[z slot + i + j ld], z in order from 0.0, as the
// reduction kernels form it (so the factorisation sees the same bits).
// (Used for the batched Gram matrices, split into at most a few chunks.)
struct GSrc {
  const double* G;
  int64_t ld;
  const double* part;
  int nz;
  int64_t slot;
  __device__ __forceinline__ double at(int i, int j) const {
    if (part == nullptr) return G[i + static_cast<int64_t>(j) * ld];
    const double* p = part + i + static_cast<int64_t>(j) * ld;
    double v = 0.0;
    for (int z = 0; z < nz; ++z) v += p[z * slot];
    return v;
  }
};
__device__ __forceinline__ GSrc gsrc(const double* G, int64_t ld) {
  return GSrc{G, ld, nullptr, 1, 0};
}

// Blocked Cholesky with dropping of the w x w matrix G (column-major, ld w).
// Result in LDS: Ts[c * TS + i] = T[c][i] = L[i][c] (T = L^T upper
// triangular, zero for i < c and in the padding up to WMAX); flag, rdiag,
// the kept list and count, and the list of dropped or padding columns.
//
// G enters scaled by 2^(2 sexp), chosen so that its largest diagonal entry
// lies in [1/2, 2) (sexp = 0 for a zero or non-finite maximum); the factor
// of the scaled matrix is 2^sexp T, and its inverse 2^-sexp T^{-1}.  Power
// of two scaling is exact and leaves every pivot test unchanged, and it
// keeps every kept pivot inside the range of the hardware reciprocal square
// root estimate.
// G: the w x w matrix factorised (GSrc).  Gd (wd x wd): the matrix whose
// largest diagonal entry fixes the power-of-two scale and the drop
// threshold; G itself for a whole Gram matrix, the whole Gram matrix when G
// is one of its diagonal blocks or a Schur complement (so every block is
// scaled and tested as the unblocked factorisation would be).
template <int WMAX, int NW>
__device__ __forceinline__ void chol_blocked(const GSrc& G, int w, const GSrc& Gd, int wd, double* Ts,
                                             int* flag, double* rdiag, int* klist, int* kcnt,
                                             int* ulist, int* ucnt, int& sexp) {
  constexpr int TS = WMAX + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double gscaled = 0.0;
  // lower triangle of G into Ts, everything else zero; every load of a
  // thread is issued before the first store.  Each wave also reads the
  // diagonal to find the scale.
  {
    constexpr int PER = WMAX * WMAX / (64 * NW);
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 64 * NW * q;
      const int i = idx % WMAX, j = idx / WMAX;
      v[q] = (i < w && j < w && i >= j) ? G.at(i, j) : 0.0;
    }
    double gd = 0.0;
    for (int c = lane; c < wd; c += 64) gd = fmax(gd, Gd.at(c, c));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) gd = fmax(gd, __shfl_xor(gd, off));
    int ex = 0;
    if (gd > 0.0 && gd <= 0x1.fffffffffffffp+1023) (void)frexp(gd, &ex);
    sexp = (gd > 0.0 && gd <= 0x1.fffffffffffffp+1023) ? ((1 - ex) >> 1) : 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 64 * NW * q;
      Ts[(idx / WMAX) * TS + idx % WMAX] = ldexp(v[q], 2 * sexp);
    }
    gscaled = ldexp(gd, 2 * sexp);  // exact: the largest scaled diagonal entry
  }
  lds_barrier();
  const double gmax = gscaled;
  const double thresh = kDropRel * gmax;
  auto panel = [&](int p) {
    if (WMAX > 64 && p + 64 < WMAX)
      chol_panel<WMAX, WMAX / 64>(Ts, p, w, thresh, gmax > 0.0, flag, rdiag);
    else
      chol_panel<WMAX, 1>(Ts, p, w, thresh, gmax > 0.0, flag, rdiag);
  };
  // Look-ahead: after panel p, all waves first update the block column of
  // the next panel; then wave 0 factors that panel while the other waves
  // finish the trailing update of panel p (blocks bj >= 1, which neither
  // read nor write the next panel's columns).
  if (wave == 0) panel(0);
  lds_barrier();
  for (int p = 0; p + kPanel < w; p += kPanel) {
    const int nb = (w - p - kPanel + 15) / 16;
    for (int bi = wave; bi < nb; bi += NW) chol_trail_block(Ts, TS, p, bi, 0);
    lds_barrier();
    if (wave == 0) {
      panel(p + kPanel);
    } else {
      const int rest = (nb - 1) * nb / 2;  // triangle of blocks with bj >= 1
      for (int job = wave - 1; job < rest; job += NW - 1) {
        int bi, bj;
        tri_index(job, bi, bj);
        chol_trail_block(Ts, TS, p, bi + 1, bj + 1);
      }
    }
    lds_barrier();
  }
  // padding columns: dropped, unit pivots
  for (int c = (w + kPanel - 1) / kPanel * kPanel + threadIdx.x; c < WMAX; c += 64 * NW) {
    flag[c] = 0;
    rdiag[c] = 1.0;
  }
  // kept list in column order (ballot + prefix count by wave 0), and the
  // list of the other columns up to WMAX (dropped or padding) after it
  if (wave == 0) {
    int base = 0, ubase = 0;
    for (int c0 = 0; c0 < WMAX; c0 += 64) {
      const int c = c0 + lane;
      const bool f = (c < w) && flag[c];
      const unsigned long long m = __ballot(f);
      const unsigned long long mu = __ballot(!f);
      const unsigned long long below = (1ull << lane) - 1ull;
      if (f) klist[base + __popcll(m & below)] = c;
      else ulist[ubase + __popcll(mu & below)] = c;
      base += __popcll(m);
      ubase += __popcll(mu);
    }
    if (lane == 0) {
      *kcnt = base;
      *ucnt = ubase;
    }
  }
  lds_barrier();
}

// ---- fused Cholesky + inverse for panels up to 128 wide -------------------
//
// T goes to LDS (row-major, odd row stride).  Dropped columns become unit
// rows and columns, T' = T_kept (+) I, whose inverse restricted to the kept
// rows and columns is T_kept^{-1}.  The inverse is formed in place:
//   * 16 x 16 diagonal blocks by back substitution, one column per lane
//     (T X = I solved from the bottom row up, register arrays with
//     compile-time indices, broadcast LDS reads of T);
//   * pairs of finished blocks joined by X_AB = -X_A (T_AB X_B), the two
//     products on v_mfma_f64_16x16x4_f64, the intermediate kept in the free
//     strictly-lower part of the LDS array.
// Output: Tinv (w x w, column-major): column a < count is column kept[a] of
// T'^{-1}; columns a >= count are zero.
template <int WMAX>
struct LdsInvShape {
  static constexpr int TS = WMAX + 1;  // LDS row stride (odd: conflict-free MFMA fragment reads)
  static constexpr int NW = 8;
  static constexpr int THREADS = 64 * NW;
};

// One 16 x 16 output block (bi, bj) of C = alpha * A B with S x S operands
// in LDS (row stride TS): A at (ra, ka), B at (kb, cb), C at (rc, cc).  The
// sum runs over the 16-deep slices [k0, k1) only; the caller passes the
// range outside which one triangular operand is zero.
template <int TS>
__device__ __forceinline__ void lds_block16(double* M, int ra, int ka, int kb, int cb, int rc,
                                            int cc, double alpha, int bi, int bj, int k0, int k1) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const double* pa = M + (ra + 16 * bi + (lane & 15)) * TS + ka + (lane >> 4);
  const double* pb = M + (kb + (lane >> 4)) * TS + cb + 16 * bj + (lane & 15);
  d4 acc = (d4){0.0, 0.0, 0.0, 0.0};
  for (int k16 = k0; k16 < k1; ++k16) {
    double a[4], b[4];
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      a[k4] = pa[16 * k16 + 4 * k4];
      b[k4] = pb[(16 * k16 + 4 * k4) * TS];
    }
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k4], b[k4], acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    M[(rc + 16 * bi + (lane >> 4) + 4 * r) * TS + cc + 16 * bj + (lane & 15)] = alpha * acc[r];
}

template <int WMAX>
__device__ __forceinline__ void chol_inv_lds_body(const GSrc& G, int w, const GSrc& Gd, int wd,
                                                  int* __restrict__ kept,
                                                  double* __restrict__ Tinv, int ldt) {
  using L = LdsInvShape<WMAX>;
  constexpr int TS = L::TS, NW = L::NW;
  __shared__ double Ts[WMAX * TS];
  __shared__ double rdiag[WMAX];
  __shared__ int flag[WMAX];
  __shared__ int klist[WMAX];
  __shared__ int ulist[WMAX];
  __shared__ int kcnt, ucnt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  int sexp;
  chol_blocked<WMAX, NW>(G, w, Gd, wd, Ts, flag, rdiag, klist, &kcnt, ulist, &ucnt, sexp);
  // T' = T with every dropped or padding index u turned into a unit row and
  // column (its inverse restricted to the kept indices is T_kept^{-1})
  const int nu = ucnt;
  if (nu > 0) {
    for (int job = wave; job < nu; job += NW) {
      const int u = ulist[job];
      for (int c = lane; c < WMAX; c += 64) {
        if (c >= u) Ts[u * TS + c] = (c == u) ? 1.0 : 0.0;
        if (c <= u) Ts[c * TS + u] = (c == u) ? 1.0 : 0.0;
      }
    }
    lds_barrier();
  }

  // 16 x 16 diagonal blocks, one per wave, lanes 0..15 one column each:
  // T X = I from the bottom row up in axpy form, with the stored pivot
  // reciprocals instead of divisions
  if (wave < WMAX / 16 && lane < 16) {
    const int o = 16 * wave, j = lane;
    double x[16];
    static_for<16>([&](auto r) { x[r] = (r == j) ? 1.0 : 0.0; });
    static_for<16>([&](auto ii) {
      constexpr int i = 15 - decltype(ii)::value;
      x[i] *= rdiag[o + i];
      static_for<i>([&](auto r) { x[r] = fma(-Ts[(o + r) * TS + o + i], x[i], x[r]); });
    });
    static_for<16>([&](auto i) { Ts[(o + i) * TS + o + j] = x[i]; });
  }
  lds_barrier();

  // join pairs of inverted s x s blocks, s = 16, 32, ...: X_AB = -X_A (T_AB X_B);
  // the 16 x 16 output blocks of all pairs of a level are spread over the waves
  static_for<(WMAX == 128) ? 3 : 2>([&](auto lev) {
    constexpr int s = 16 << decltype(lev)::value;
    constexpr int pairs = WMAX / (2 * s);
    constexpr int nb = s / 16;
    constexpr int jobs = pairs * nb * nb;
    // jobs are dealt in snake order (every other round reversed) so that
    // each wave gets a long and a short triangular sum
    auto job_at = [&](int j) {
      const int t = j / NW, i = j % NW;
      return (t & 1) ? t * NW + (NW - 1 - i) : j;
    };
    // M = T_AB X_B, stored at rows [ob, ob + s), columns [oa, oa + s);
    // X_B is upper triangular, so slice k of column block bj needs k <= bj
    for (int j = wave; j < jobs; j += NW) {
      const int job = job_at(j);
      const int pr = job / (nb * nb), q = job % (nb * nb);
      const int oa = 2 * s * pr, ob = oa + s;
      lds_block16<TS>(Ts, oa, ob, ob, ob, ob, oa, 1.0, q / nb, q % nb, 0, q % nb + 1);
    }
    lds_barrier();
    // X_AB = -X_A M over T_AB: A = X_A at (oa, oa), B = M at (ob, oa);
    // X_A is upper triangular, so row block bi needs slices k >= bi
    for (int j = wave; j < jobs; j += NW) {
      const int job = job_at(j);
      const int pr = job / (nb * nb), q = job % (nb * nb);
      const int oa = 2 * s * pr, ob = oa + s;
      lds_block16<TS>(Ts, oa, oa, ob, oa, oa, ob, -1.0, q / nb, q % nb, q / nb, nb);
    }
    lds_barrier();
    // clear M: the joined 2s x 2s block must be upper triangular again
    for (int idx = threadIdx.x; idx < pairs * s * s; idx += blockDim.x) {
      const int pr = idx / (s * s), e = idx % (s * s);
      const int oa = 2 * s * pr, ob = oa + s;
      Ts[(ob + e / s) * TS + oa + e % s] = 0.0;
    }
    lds_barrier();
  });

  // expanded inverse: column a <- column kept[a] of T'^{-1} (undoing the
  // scale of G), zero for a >= count
  const int wk = kcnt;
  for (int a = wave; a < w; a += NW) {
    double* col = Tinv + static_cast<int64_t>(a) * ldt;
    if (a < wk) {
      const int kc = klist[a];
      for (int r = lane; r < w; r += 64) col[r] = ldexp(Ts[r * TS + kc], sexp);
    } else {
      for (int r = lane; r < w; r += 64) col[r] = 0.0;
    }
  }
  for (int i = threadIdx.x; i < wk; i += blockDim.x) kept[1 + i] = klist[i];
  if (threadIdx.x == 0) kept[0] = wk;
}

template <int WMAX>
__global__ __launch_bounds__(512) void chol_inv_lds_kernel(const double* __restrict__ G, int w,
                                                           int* __restrict__ kept,
                                                           double* __restrict__ Tinv) {
  chol_inv_lds_body<WMAX>(gsrc(G, w), w, gsrc(G, w), w, kept, Tinv, w);
}

// one diagonal block (or Schur complement) of a wider Gram matrix Gd
template <int WMAX>
__global__ __launch_bounds__(512) void chol_inv_block_kernel(const double* __restrict__ G, int w,
                                                             int ldg, const double* __restrict__ Gd,
                                                             int wd, int* __restrict__ kept,
                                                             double* __restrict__ Tinv, int ldt) {
  chol_inv_lds_body<WMAX>(gsrc(G, ldg), w, gsrc(Gd, wd), wd, kept, Tinv, ldt);
}

// one workgroup per problem of a batch
template <int WMAX>
__global__ __launch_bounds__(512) void chol_inv_batched_kernel(const BatchChol* __restrict__ desc) {
  const BatchChol c = desc[blockIdx.x];
  if (c.w <= 0) return;  // a problem that takes no part in this step
  const GSrc g = c.ksplit > 1 ? GSrc{nullptr, c.ldp, c.part, c.ksplit, c.slot} : gsrc(c.G, c.w);
  chol_inv_lds_body<WMAX>(g, c.w, g, c.w, c.kept, c.Tinv, c.w);
}

template <int WMAX>
int launch_chol_inv_lds(const double* G, int w, int* kept, double* Tinv, hipStream_t s) {
  ProfScope ps(kKChol, 2.0 * double(w) * w * w / 3.0, 16.0 * w * w, s);
  hipLaunchKernelGGL(chol_inv_lds_kernel<WMAX>, dim3(1), dim3(LdsInvShape<WMAX>::THREADS), 0, s,
                     G, w, kept, Tinv);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

// S = G22 - M (w2 x w2): the Schur complement of the leading 128 x 128
// block, G22 the trailing block of G (ld ldg), M = T12^T T12 (ld w2)
__global__ __launch_bounds__(256) void schur_kernel(const double* __restrict__ G, int ldg, int h,
                                                    int w2, const double* __restrict__ M,
                                                    double* __restrict__ S) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= w2 * w2) return;
  const int i = idx % w2, j = idx / w2;
  S[idx] = G[(h + i) + static_cast<int64_t>(h + j) * ldg] - M[idx];
}

// Assemble T^{-1} (w x w, kept columns first) from the two blocks:
// columns [0, k1): the first block's inverse in rows [0, h), zero below;
// columns [k1, k1 + k2): U (rows [0, h)) over the second block's inverse
// (rows [h, w)); zero after.  Merges the kept lists (second block offset by
// h).  One workgroup per output column c (w of them); the first also
// writes the kept list.
__global__ __launch_bounds__(256) void chol_join_kernel(int w, int h, const int* __restrict__ kept1,
                                                        const int* __restrict__ kept2,
                                                        const double* __restrict__ U,
                                                        const double* __restrict__ T22inv,
                                                        double* __restrict__ Tinv,
                                                        int* __restrict__ kept) {
  const int k1 = kept1[0], k2 = kept2[0], w2 = w - h;
  const int c = blockIdx.x;
  double* col = Tinv + static_cast<int64_t>(c) * w;
  if (c < k1) {
    for (int r = h + threadIdx.x; r < w; r += 256) col[r] = 0.0;
  } else {
    const int a = c - k1;
    for (int r = threadIdx.x; r < w; r += 256)
      col[r] = a >= k2 ? 0.0 : (r < h ? U[r + a * h] : T22inv[(r - h) + a * w2]);
  }
  if (c == 0) {
    for (int i = threadIdx.x; i < k1 + k2; i += 256)
      kept[1 + i] = i < k1 ? kept1[1 + i] : h + kept2[1 + (i - k1)];
    if (threadIdx.x == 0) kept[0] = k1 + k2;
  }
}

// Panels of 129..256 columns, blocked 128 + (w - 128) (G = T^T T, T upper):
//   T11 from the LDS kernel on G11 (T11^{-1} into Tinv's leading block),
//   T12 = T11^{-T} G12,  S = G22 - T12^T T12,  T22 from the LDS kernel on S,
//   upper-right block of T^{-1}:  U = -T11^{-1} (T12 T22^{-1}),
// with the power-of-two scale and the drop threshold of the whole G in both
// factorisations: the pivots of S are those the unblocked factorisation
// meets for columns 128.., so the same columns are kept.  scratch: 6 h^2
// doubles and 2 (h + 1) ints after them.
int chol_inv_wide(const double* G, int w, double* scratch, int* kept, double* Tinv,
                  hipStream_t s) {
  constexpr int h = 128;
  const int w2 = w - h;
  double* T12 = scratch;            // h x w2, ld h
  double* M = T12 + h * h;          // w2 x w2
  double* S = M + h * h;            // w2 x w2
  double* T22inv = S + h * h;       // w2 x w2
  double* W = T22inv + h * h;       // h x w2
  double* U = W + h * h;            // h x w2
  int* kept1 = reinterpret_cast<int*>(U + h * h);
  int* kept2 = kept1 + h + 1;
  {
    ProfScope ps(kKChol, 2.0 * double(w) * w * w / 3.0, 16.0 * w * w, s);
    hipLaunchKernelGGL(chol_inv_block_kernel<128>, dim3(1), dim3(LdsInvShape<128>::THREADS), 0, s,
                       G, h, w, G, w, kept1, Tinv, w);
  }
  QB_HIP_TRY(hipGetLastError());
  int rc = gemm_tn(Tinv, w, G + static_cast<int64_t>(h) * w, w, T12, h, h, w2, h, false, 1,
                   nullptr, nullptr, nullptr, s);
  if (rc) return rc;
  rc = gemm_tn(T12, h, T12, h, M, w2, w2, w2, h, false, 1, nullptr, nullptr, nullptr, s);
  if (rc) return rc;
  hipLaunchKernelGGL(schur_kernel, dim3(static_cast<unsigned>((w2 * w2 + 255) / 256)), dim3(256),
                     0, s, G, w, h, w2, M, S);
  QB_HIP_TRY(hipGetLastError());
  {
    ProfScope ps(kKChol, 0.0, 0.0, s);
    hipLaunchKernelGGL(chol_inv_block_kernel<128>, dim3(1), dim3(LdsInvShape<128>::THREADS), 0, s,
                       S, w2, w2, G, w, kept2, T22inv, w2);
  }
  QB_HIP_TRY(hipGetLastError());
  rc = gemm_nn(T12, h, T22inv, w2, W, h, h, w2, w2, 1.0, 0.0, 1, nullptr, s);
  if (rc) return rc;
  rc = gemm_nn(Tinv, w, W, h, U, h, h, w2, h, -1.0, 0.0, 1, nullptr, s);
  if (rc) return rc;
  hipLaunchKernelGGL(chol_join_kernel, dim3(static_cast<unsigned>(w)), dim3(256), 0, s, w, h,
                     kept1, kept2, U, T22inv, Tinv, kept);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int chol_inv(const double* G, int w, double* T, int* kept, double* Tinv, hipStream_t s) {
  if (w <= 64) return launch_chol_inv_lds<64>(G, w, kept, Tinv, s);
  if (w <= 128) return launch_chol_inv_lds<128>(G, w, kept, Tinv, s);
  if (w <= 256) return chol_inv_wide(G, w, T, kept, Tinv, s);
  return kEInval;
}

// one pass: Qout = X_kept T^{-1}.  The Gram matrix is summed from its
// depth chunks by the reduction kernel before the Cholesky: at m = 10^4 it
// has about 63 chunks, and summing them inside the one-workgroup Cholesky
// as it loads G (a chain of dependent loads per element) took 12 times as
// long as the reduction it saves.
int cholqr_pass(const double* X, int64_t ldx, double* Qout, int64_t ldqo, int64_t m, int w,
                const OrthWork& ow, hipStream_t s) {
  int rc = gemm_tn(X, ldx, X, ldx, ow.gram, w, w, w, m, false, ow.split, ow.part, nullptr,
                   nullptr, s);
  if (rc) return rc;
  rc = chol_inv(ow.gram, w, ow.tfull, ow.kept, ow.tinv, s);
  if (rc) return rc;
  return gemm_nn(X, ldx, ow.tinv, w, Qout, ldqo, m, w, w, 1.0, 0.0, 1, nullptr, s);
}

}  // namespace

int chol_inv_batched(const BatchChol* desc, int count, hipStream_t s) {
  if (count <= 0) return kOk;
  ProfScope ps(kKCholBatched, 0.0, 0.0, s);
  hipLaunchKernelGGL(chol_inv_batched_kernel<64>, dim3(static_cast<unsigned>(count)),
                     dim3(LdsInvShape<64>::THREADS), 0, s, desc);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

size_t orth_work_bytes(int64_t m, int w) {
  Arena a{nullptr, 0, 0};
  OrthWork ow;
  orth_carve(a, m, w, &ow);
  return a.used + 256;
}

int orth_carve(Arena& a, int64_t m, int w, OrthWork* ow) {
  ow->ldt = (m + 1) & ~int64_t(1);
  ow->gram = a.take<double>(static_cast<size_t>(w) * w);
  // scratch of chol_inv_wide (panels wider than 128)
  ow->tfull = a.take<double>(w > 128 ? std::max(static_cast<size_t>(w) * w,
                                                static_cast<size_t>(6 * 128 * 128 + 2 * 129))
                                     : static_cast<size_t>(w) * w);
  ow->tinv = a.take<double>(static_cast<size_t>(w) * w);
  ow->qtmp = a.take<double>(static_cast<size_t>(ow->ldt) * w);
  ow->kept = a.take<int>(static_cast<size_t>(w) + 1);
  // The Gram runs on 64 x 64 tiles.  For panels up to 128 wide, a single
  // round with at most one workgroup per CU was measured fastest (w = 128,
  // m = 10^4: 16.9 us for product and reduce at 4 x 63 workgroups, 20.3 us
  // at 4 x 70).
  ow->split = choose_split(w, w, m);
  const int gt = ((w + 63) / 64) * ((w + 63) / 64);
  if (gt <= 4 && ow->split > kNumCU / gt) ow->split = kNumCU / gt;
  ow->part = a.take<double>(partial_doubles(w, w, ow->split) + 1);
  return (a.base != nullptr && a.used > a.cap) ? kEWorkspace : kOk;
}

int orth_cholqr2(const double* X, int64_t ldx, double* Q, int64_t ldq, int64_t m, int w,
                 const OrthWork& ow, hipStream_t s) {
  if (w < 1 || w > kMaxPanel) return kEInval;
  int rc = cholqr_pass(X, ldx, ow.qtmp, ow.ldt, m, w, ow, s);
  if (rc) return rc;
  return cholqr_pass(ow.qtmp, ow.ldt, Q, ldq, m, w, ow, s);
}

namespace {
// flag[0] = 1 when a pass kept fewer than w columns
__global__ void flag_dropped_kernel(const int* __restrict__ kept, int w, int* __restrict__ flag) {
  if (threadIdx.x == 0 && kept[0] != w) flag[0] = 1;
}
}  // namespace

int orth_cholqr2_rinv(const double* X, int64_t ldx, double* Q, int64_t ldq, int64_t m, int w,
                      const OrthWork& ow, double* t1inv, double* rinv, int* dropped,
                      hipStream_t s) {
  if (w < 1 || w > kMaxPanel) return kEInval;
  int rc = cholqr_pass(X, ldx, ow.qtmp, ow.ldt, m, w, ow, s);
  if (rc) return rc;
  hipLaunchKernelGGL(flag_dropped_kernel, dim3(1), dim3(64), 0, s, ow.kept, w, dropped);
  QB_HIP_TRY(hipGetLastError());
  rc = copy_matrix(ow.tinv, w, t1inv, w, w, w, s);
  if (rc) return rc;
  rc = cholqr_pass(ow.qtmp, ow.ldt, Q, ldq, m, w, ow, s);
  if (rc) return rc;
  hipLaunchKernelGGL(flag_dropped_kernel, dim3(1), dim3(64), 0, s, ow.kept, w, dropped);
  QB_HIP_TRY(hipGetLastError());
  // R = T2 T1, so R^{-1} = T1^{-1} T2^{-1}
  return gemm_nn(t1inv, w, ow.tinv, w, rinv, w, w, w, w, 1.0, 0.0, 1, nullptr, s);
}

}  // namespace qb
