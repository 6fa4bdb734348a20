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
// Cholesky: one workgroup, the lower triangle of G held in registers.  Row i
// of G lives in lane i % 64 (slot i / 64), column j in wave j % NW (slot
// j / NW).  Column c is finished by its owning wave alone (a lane shuffle
// broadcasts the pivot), written to a double-buffered LDS row, and after a
// single barrier every thread applies the rank-one update to the part of
// the trailing matrix it holds.  One barrier per column.
//
// Inverse: T^{-1} of the kept part, one workgroup (one wave) per output
// column, by back substitution in column-oriented form.
#include <utility>

#include "qb_internal.hpp"

namespace qb {
namespace {

constexpr double kDropRel = 0x1p-40;

// WMAX: widest panel handled; NW: waves (must divide 64).  A thread holds
// the lower-triangle entries of its (row slot, column slot) pairs.
template <int WMAX, int NW_>
struct CholShape {
  static constexpr int NW = NW_;          // waves
  static constexpr int RA = WMAX / 64;    // row slots per lane
  static constexpr int CB = WMAX / NW_;   // column slots per wave
  static constexpr int THREADS = 64 * NW_;
  static constexpr bool valid(int a, int bb) { return 64 * a + 63 >= NW * bb; }
};

// compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int WMAX, int NW_>
__global__ __launch_bounds__(64 * NW_) void chol_drop_kernel(
    const double* __restrict__ G, int w, double* __restrict__ T, int* __restrict__ kept) {
  using S = CholShape<WMAX, NW_>;
  constexpr int NW = S::NW, RA = S::RA, CB = S::CB;
  __shared__ double lbuf[2][WMAX];
  __shared__ double dsh[WMAX];
  __shared__ int flag[WMAX];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;

  double g[RA][CB];
  static_for<RA>([&](auto a) {
    static_for<CB>([&](auto bb) {
      if constexpr (S::valid(a, bb)) {
        const int i = lane + 64 * a, j = wave + NW * bb;
        g[a][bb] = (i < w && j < w && i >= j) ? G[i + static_cast<int64_t>(j) * w] : 0.0;
        if (i == j && i < w) dsh[i] = g[a][bb];
      }
    });
  });
  __syncthreads();
  double gmax = 0.0;
  for (int c = 0; c < w; ++c) gmax = fmax(gmax, dsh[c]);
  const double thresh = kDropRel * gmax;

  static_for<CB>([&](auto cb) {
    constexpr int ac = (NW * cb) / 64;  // row slot holding the diagonal of this column slot
    for (int W = 0; W < NW; ++W) {
      const int c = W + NW * cb;
      if (c >= w) break;
      double* buf = lbuf[c & 1];
      if (wave == W) {
        double gd = 0.0;
        if constexpr (S::valid(ac, cb)) gd = g[ac][cb];
        const double d = __shfl(gd, c & 63);
        const bool keep = (d > thresh) && (gmax > 0.0);
        const double sdiag = keep ? sqrt(d) : 0.0;
        const double inv = keep ? 1.0 / sdiag : 0.0;
        static_for<RA>([&](auto a) {
          const int i = lane + 64 * a;
          double v = 0.0;
          if constexpr (S::valid(a, cb)) v = (i > c) ? g[a][cb] * inv : 0.0;
          if (i == c) v = sdiag;
          buf[i] = v;
          if (i < w) T[c + static_cast<int64_t>(i) * w] = (i >= c) ? v : 0.0;
        });
        if (lane == 0) flag[c] = keep ? 1 : 0;
      }
      __syncthreads();
      double rv[RA];
      static_for<RA>([&](auto a) { rv[a] = buf[lane + 64 * a]; });
      static_for<CB>([&](auto bb) {
        const int j = wave + NW * bb;
        if (j > c) {
          const double cvb = buf[j];
          static_for<RA>([&](auto a) {
            if constexpr (S::valid(a, bb)) {
              const int i = lane + 64 * a;
              if (i >= j) g[a][bb] -= rv[a] * cvb;
            }
          });
        }
      });
    }
  });
  __syncthreads();
  if (threadIdx.x == 0) {
    int cnt = 0;
    for (int c = 0; c < w; ++c)
      if (flag[c]) kept[1 + cnt++] = c;
    kept[0] = cnt;
  }
}

// Column `a` of the inverse of the kept part Tc = T[kept][:, kept]; written
// into Tinv (w x w) at rows kept[i], zero elsewhere and for a >= count.
template <int WMAX>
__global__ __launch_bounds__(64) void trinv_kernel(const double* __restrict__ T, int w,
                                                   const int* __restrict__ kept,
                                                   double* __restrict__ Tinv) {
  constexpr int RA = WMAX / 64;
  __shared__ int kidx[WMAX];
  const int a = blockIdx.x;
  const int lane = threadIdx.x;
  const int wk = kept[0];
  double* out = Tinv + static_cast<int64_t>(a) * w;
  for (int i = lane; i < w; i += 64) out[i] = 0.0;
  if (a >= wk) return;
  for (int i = lane; i < wk; i += 64) kidx[i] = kept[1 + i];
  __syncthreads();
  double s[RA];
  int64_t rowoff[RA];
#pragma unroll
  for (int q = 0; q < RA; ++q) {
    const int i = lane + 64 * q;
    s[q] = (i == a) ? 1.0 : 0.0;
    rowoff[q] = (i < wk) ? kidx[i] : 0;
  }
  int kl = kidx[a];
  double tcol[RA];
#pragma unroll
  for (int q = 0; q < RA; ++q) tcol[q] = T[rowoff[q] + static_cast<int64_t>(kl) * w];
  for (int l = a; l >= 0; --l) {
    // prefetch the next column while this one is applied
    double tnext[RA];
    const int kn = (l > 0) ? kidx[l - 1] : kl;
#pragma unroll
    for (int q = 0; q < RA; ++q) tnext[q] = T[rowoff[q] + static_cast<int64_t>(kn) * w];
    double own = 0.0, tll = 0.0;
#pragma unroll
    for (int q = 0; q < RA; ++q)
      if (q == (l >> 6)) { own = s[q]; tll = tcol[q]; }
    const double sl = __shfl(own, l & 63);
    const double dl = __shfl(tll, l & 63);
    const double xl = sl / dl;
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int i = lane + 64 * q;
      if (i < l) s[q] -= tcol[q] * xl;
      if (i == l) s[q] = xl;
    }
#pragma unroll
    for (int q = 0; q < RA; ++q) tcol[q] = tnext[q];
    kl = kn;
  }
#pragma unroll
  for (int q = 0; q < RA; ++q) {
    const int i = lane + 64 * q;
    if (i <= a) out[rowoff[q]] = s[q];
  }
}

template <int WMAX, int NW>
int launch_chol_inv(const double* G, int w, double* T, int* kept, double* Tinv, hipStream_t s) {
  const double w3 = double(w) * w * w / 3.0, w2b = 16.0 * w * w;
  {
    ProfScope ps(kKChol, w3, w2b, s);
    hipLaunchKernelGGL((chol_drop_kernel<WMAX, NW>), dim3(1), dim3(CholShape<WMAX, NW>::THREADS),
                       0, s, G, w, T, kept);
  }
  QB_HIP_TRY(hipGetLastError());
  {
    ProfScope ps(kKTrinv, w3, w2b, s);
    hipLaunchKernelGGL(trinv_kernel<WMAX>, dim3(static_cast<unsigned>(w)), dim3(64), 0, s, T, w,
                       kept, Tinv);
  }
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int chol_inv(const double* G, int w, double* T, int* kept, double* Tinv, hipStream_t s) {
  if (w <= 64) return launch_chol_inv<64, 4>(G, w, T, kept, Tinv, s);
  if (w <= 128) return launch_chol_inv<128, 8>(G, w, T, kept, Tinv, s);
  if (w <= 256) return launch_chol_inv<256, 8>(G, w, T, kept, Tinv, s);
  return kEInval;
}

// one pass: Qout = X_kept T^{-1}
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

size_t orth_work_bytes(int64_t m, int w) {
  Arena a{nullptr, 0, 0};
  OrthWork ow;
  orth_carve(a, m, w, &ow);
  return a.used + 256;
}

int orth_carve(Arena& a, int64_t m, int w, OrthWork* ow) {
  ow->ldt = (m + 1) & ~int64_t(1);
  ow->gram = a.take<double>(static_cast<size_t>(w) * w);
  ow->tfull = a.take<double>(static_cast<size_t>(w) * w);
  ow->tinv = a.take<double>(static_cast<size_t>(w) * w);
  ow->qtmp = a.take<double>(static_cast<size_t>(ow->ldt) * w);
  ow->kept = a.take<int>(static_cast<size_t>(w) + 1);
  ow->split = choose_split(w, w, m);
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

}  // namespace qb
