// Standard factorisations from A ~ Q B (Section 3.3).
//
// Low-rank SVD (Section 3.3.1).  The SVD of the k x n matrix B comes from
// one-sided (Hestenes) Jacobi on B^T: plane rotations J applied to pairs
// of columns of B^T until all columns are mutually orthogonal, so that
// B^T J = W with orthogonal columns.  Then B = J Sigma (W Sigma^-1)^T:
// the left singular vectors of B are the columns of J, the right ones the
// normalised columns of W, and U = Q J.  Rotating the columns directly
// keeps the high relative accuracy of the small singular values that a
// Gram-matrix route would lose below sqrt(u) sigma_1.  One round applies
// K/2 disjoint rotations (round-robin pairing, K = k rounded up to even),
// one workgroup per pair; K - 1 rounds make a sweep; sweeps repeat until
// every pair is orthogonal to a relative 1e-15.  The singular values are
// then sorted in one workgroup (bitonic, ties by index) and U = Q J on the
// MFMA GEMM.
//
// Partial pivoted QR (Section 3.3.2).  B P = Q_tilde R by Householder QR
// with column pivoting: at step j the remaining column of largest norm
// (rows j.., recomputed exactly every step, ties to the smallest index) is
// swapped to position j and reflected onto beta e_1, beta = -sign(x_0) ||x||.
// One step is two launches: a single workgroup selects the pivot, swaps and
// forms the reflector; then one wave per trailing column applies it and
// computes that column's norm for the next step, with per-workgroup argmax
// candidates.  Q_tilde is accumulated backwards on the identity (k x k),
// then Q_hat = Q Q_tilde on the MFMA GEMM.
//
// Every reduction has a fixed order: results are bitwise reproducible.
#include <algorithm>
#include <cmath>

#include "../../include/qb.h"
#include "qb_internal.hpp"

namespace qb {
namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t even_up(int64_t v) { return (v + 1) & ~int64_t(1); }

constexpr int kJacThreads = 256;
constexpr int kMaxSweeps = 60;
constexpr double kJacTol = 1e-15;
constexpr int kSortThreads = 1024;
constexpr int kSortMax = 4096;   // largest k the one-workgroup sort takes

// ---- Bt (n x k, ldt) = B^T, B (k x n, ldb); 32 x 32 tiles through LDS --
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ B, int64_t ldb,
                                                        double* __restrict__ Bt, int64_t ldt,
                                                        int64_t k, int64_t n) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t i0 = static_cast<int64_t>(blockIdx.y) * 32;  // rows of B
  const int64_t j0 = static_cast<int64_t>(blockIdx.x) * 32;  // columns of B
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + tx, j = j0 + r;
    tile[r][tx] = (i < k && j < n) ? B[i + j * ldb] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + tx, i = i0 + r;
    if (j < n && i < k) Bt[j + i * ldt] = tile[tx][r];
  }
}

__global__ __launch_bounds__(256) void identity_kernel(double* __restrict__ X, int64_t ld, int k) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(k) * k) return;
  const int64_t i = idx % k, j = idx / k;
  X[i + j * ld] = (i == j) ? 1.0 : 0.0;
}

// fixed-order sum over a 256-thread workgroup; every thread gets the total
__device__ __forceinline__ double block_sum256(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// column of position p in round r of the round-robin pairing of K columns
__device__ __forceinline__ int rr_index(int p, int r, int K) {
  return p == 0 ? 0 : 1 + (p - 1 + r) % (K - 1);
}

// One Jacobi round: workgroup i rotates the pair (a, b) of round r.
// offmax[i] keeps the largest relative off-diagonal |x.y|/(|x||y|) seen by
// this pair slot during the sweep.
__global__ __launch_bounds__(kJacThreads) void jacobi_round_kernel(
    double* __restrict__ Bt, int64_t ldt, int64_t n, double* __restrict__ J, int64_t ldj, int k,
    int K, int r, double* __restrict__ offmax) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  int a = rr_index(i, r, K), b = rr_index(K - 1 - i, r, K);
  if (a > b) { const int t = a; a = b; b = t; }
  if (b >= k) return;  // the padding column of an odd k
  double* x = Bt + static_cast<int64_t>(a) * ldt;
  double* y = Bt + static_cast<int64_t>(b) * ldt;
  double sa = 0.0, sb = 0.0, sg = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += kJacThreads) {
    const double xa = x[t], yb = y[t];
    sa = fma(xa, xa, sa);
    sb = fma(yb, yb, sb);
    sg = fma(xa, yb, sg);
  }
  const double alpha = block_sum256(sa, red);
  const double beta = block_sum256(sb, red);
  const double gamma = block_sum256(sg, red);
  double off = 0.0;
  if (alpha > 0.0 && beta > 0.0) off = fabs(gamma) / (sqrt(alpha) * sqrt(beta));
  if (threadIdx.x == 0) offmax[i] = fmax(offmax[i], off);
  if (!(off > kJacTol)) return;
  // rotation [x y] <- [x y] [[c, s], [-s, c]] making x and y orthogonal
  const double zeta = (beta - alpha) / (2.0 * gamma);
  const double az = fabs(zeta);
  const double tt = (az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az)));
  const double t = zeta >= 0.0 ? tt : -tt;
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  for (int64_t q = threadIdx.x; q < n; q += kJacThreads) {
    const double xa = x[q], yb = y[q];
    x[q] = c * xa - s * yb;
    y[q] = s * xa + c * yb;
  }
  double* ja = J + static_cast<int64_t>(a) * ldj;
  double* jb = J + static_cast<int64_t>(b) * ldj;
  for (int q = threadIdx.x; q < k; q += kJacThreads) {
    const double xa = ja[q], yb = jb[q];
    ja[q] = c * xa - s * yb;
    jb[q] = s * xa + c * yb;
  }
}

__global__ __launch_bounds__(256) void zero_kernel1(double* __restrict__ x, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// largest entry of x[0..n) into out[0] (one workgroup, fixed order)
__global__ __launch_bounds__(256) void max_kernel(const double* __restrict__ x, int64_t n,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, x[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// sigma_j = ||Bt(:, j)||, then a bitonic sort (descending sigma, ascending
// index on ties) of the k pairs in LDS; writes S and the order.
__global__ __launch_bounds__(kSortThreads) void sigma_sort_kernel(const double* __restrict__ Bt,
                                                                  int64_t ldt, int64_t n, int k,
                                                                  double* __restrict__ S,
                                                                  int* __restrict__ order) {
  __shared__ double key[kSortMax];
  __shared__ int idx[kSortMax];
  int P = 1;
  while (P < k) P <<= 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NWV = kSortThreads / 64;
  for (int j = wave; j < P; j += NWV) {
    double s = 0.0;
    if (j < k) {
      const double* col = Bt + static_cast<int64_t>(j) * ldt;
      for (int64_t t = lane; t < n; t += 64) s = fma(col[t], col[t], s);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    }
    if (lane == 0) {
      key[j] = (j < k) ? sqrt(s) : -1.0;
      idx[j] = j;
    }
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P; t += kSortThreads) {
        const int u = t ^ stride;
        if (u > t) {
          // "before" = larger key, then smaller index
          const bool tb = key[t] > key[u] || (key[t] == key[u] && idx[t] < idx[u]);
          const bool desc = (t & size) == 0;  // this run is sorted "before"-first
          if (desc != tb) {
            const double kk = key[t];
            key[t] = key[u];
            key[u] = kk;
            const int ii = idx[t];
            idx[t] = idx[u];
            idx[u] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < k; j += kSortThreads) {
    S[j] = key[j];
    order[j] = idx[j];
  }
}

// V(:, j) = Bt(:, order[j]) / S[j] (zero when S[j] = 0); Js(:, j) = J(:, order[j])
__global__ __launch_bounds__(256) void gather_kernel(const double* __restrict__ Bt, int64_t ldt,
                                                     int64_t n, const double* __restrict__ J,
                                                     int64_t ldj, int k,
                                                     const double* __restrict__ S,
                                                     const int* __restrict__ order,
                                                     double* __restrict__ V, int64_t ldv,
                                                     double* __restrict__ Js) {
  const int j = blockIdx.x;
  const int src = order[j];
  const double s = S[j];
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  const double* col = Bt + static_cast<int64_t>(src) * ldt;
  double* vout = V + static_cast<int64_t>(j) * ldv;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) vout[t] = col[t] * inv;
  const double* jc = J + static_cast<int64_t>(src) * ldj;
  double* jo = Js + static_cast<int64_t>(j) * ldj;
  for (int t = threadIdx.x; t < k; t += blockDim.x) jo[t] = jc[t];
}

// ---- pivoted QR ----------------------------------------------------------
constexpr int kQrCols = 4;  // columns (one wave each) per workgroup

// norms of columns [j0, n) over rows [r0, k) and per-workgroup argmax
// candidates (value, index), ties to the smaller index
__global__ __launch_bounds__(64 * kQrCols) void qr_norms_kernel(const double* __restrict__ W,
                                                               int64_t ldw, int k, int64_t n,
                                                               int r0, int64_t j0,
                                                               double* __restrict__ cval,
                                                               int64_t* __restrict__ cidx) {
  __shared__ double bv[kQrCols];
  __shared__ int64_t bi[kQrCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t col = j0 + static_cast<int64_t>(blockIdx.x) * kQrCols + wave;
  double s = -1.0;
  if (col < n) {
    const double* c = W + col * ldw;
    double acc = 0.0;
    for (int t = r0 + lane; t < k; t += 64) acc = fma(c[t], c[t], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    s = acc;
  }
  if (lane == 0) {
    bv[wave] = s;
    bi[wave] = col;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = bv[0];
    int64_t id = bi[0];
    for (int w = 1; w < kQrCols; ++w)
      if (bv[w] > v) { v = bv[w]; id = bi[w]; }
    cval[blockIdx.x] = v;
    cidx[blockIdx.x] = id;
  }
}

// Step j, one workgroup: pivot = argmax of the candidates; swap it with
// column j (W and perm); reflector of W(j:k, j) into vstore(:, j), tau[j];
// W(j, j) = beta, W(j+1:k, j) = 0.
__global__ __launch_bounds__(256) void qr_pivot_kernel(double* __restrict__ W, int64_t ldw, int k,
                                                      int j, const double* __restrict__ cval,
                                                      const int64_t* __restrict__ cidx, int ncand,
                                                      int64_t* __restrict__ perm,
                                                      double* __restrict__ vstore, int64_t ldv,
                                                      double* __restrict__ tau) {
  __shared__ double red[4];
  __shared__ int64_t piv;
  if (threadIdx.x == 0) {
    double v = cval[0];
    int64_t id = cidx[0];
    for (int c = 1; c < ncand; ++c)
      if (cval[c] > v) { v = cval[c]; id = cidx[c]; }
    piv = id;
  }
  __syncthreads();
  const int64_t p = piv;
  double* cj = W + static_cast<int64_t>(j) * ldw;
  if (p != j) {
    double* cp = W + p * ldw;
    for (int t = threadIdx.x; t < k; t += 256) {
      const double u = cj[t];
      cj[t] = cp[t];
      cp[t] = u;
    }
    if (threadIdx.x == 0) {
      const int64_t u = perm[j];
      perm[j] = perm[p];
      perm[p] = u;
    }
    __syncthreads();
  }
  double acc = 0.0;
  for (int t = j + threadIdx.x; t < k; t += 256) acc = fma(cj[t], cj[t], acc);
  const double nrm = sqrt(block_sum256(acc, red));
  const double x0 = cj[j];
  double* v = vstore + static_cast<int64_t>(j) * ldv;
  if (nrm == 0.0) {
    for (int t = j + threadIdx.x; t < k; t += 256) v[t] = (t == j) ? 1.0 : 0.0;
    if (threadIdx.x == 0) tau[j] = 0.0;
    return;
  }
  const double beta = x0 >= 0.0 ? -nrm : nrm;
  const double inv = 1.0 / (x0 - beta);
  __syncthreads();
  for (int t = j + threadIdx.x; t < k; t += 256) {
    v[t] = (t == j) ? 1.0 : cj[t] * inv;
    cj[t] = (t == j) ? beta : 0.0;
  }
  if (threadIdx.x == 0) tau[j] = (beta - x0) / beta;
}

// Apply H_j = I - tau v v^T to columns (j, n) of W (rows j..k), one wave per
// column, and leave that column's norm over rows j+1.. with per-workgroup
// argmax candidates for step j + 1.
__global__ __launch_bounds__(64 * kQrCols) void qr_apply_kernel(double* __restrict__ W, int64_t ldw,
                                                               int k, int64_t n, int j,
                                                               const double* __restrict__ vstore,
                                                               int64_t ldv,
                                                               const double* __restrict__ tau,
                                                               double* __restrict__ cval,
                                                               int64_t* __restrict__ cidx) {
  __shared__ double bv[kQrCols];
  __shared__ int64_t bi[kQrCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t col = j + 1 + static_cast<int64_t>(blockIdx.x) * kQrCols + wave;
  const double tj = tau[j];
  const double* v = vstore + static_cast<int64_t>(j) * ldv;
  double s = -1.0;
  if (col < n) {
    double* c = W + col * ldw;
    double d = 0.0;
    for (int t = j + lane; t < k; t += 64) d = fma(v[t], c[t], d);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
    const double f = tj * d;
    double acc = 0.0;
    for (int t = j + lane; t < k; t += 64) {
      const double u = c[t] - f * v[t];
      c[t] = u;
      if (t > j) acc = fma(u, u, acc);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    s = acc;
  }
  if (lane == 0) {
    bv[wave] = s;
    bi[wave] = col;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v0 = bv[0];
    int64_t id = bi[0];
    for (int w = 1; w < kQrCols; ++w)
      if (bv[w] > v0) { v0 = bv[w]; id = bi[w]; }
    cval[blockIdx.x] = v0;
    cidx[blockIdx.x] = id;
  }
}

// Qt(j:k, :) -= tau_j v_j (v_j^T Qt(j:k, :)), one wave per column of Qt
__global__ __launch_bounds__(64 * kQrCols) void qr_accum_kernel(double* __restrict__ Qt, int64_t ldq,
                                                               int k, int j,
                                                               const double* __restrict__ vstore,
                                                               int64_t ldv,
                                                               const double* __restrict__ tau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * kQrCols + wave;
  const double tj = tau[j];
  if (col >= k || tj == 0.0) return;
  const double* v = vstore + static_cast<int64_t>(j) * ldv;
  double* c = Qt + static_cast<int64_t>(col) * ldq;
  double d = 0.0;
  for (int t = j + lane; t < k; t += 64) d = fma(v[t], c[t], d);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
  const double f = tj * d;
  for (int t = j + lane; t < k; t += 64) c[t] -= f * v[t];
}

// R (k x n, ldr) = upper trapezoid of W
__global__ __launch_bounds__(256) void triu_copy_kernel(const double* __restrict__ W, int64_t ldw,
                                                        double* __restrict__ R, int64_t ldr, int k,
                                                        int64_t n) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(k) * n) return;
  const int64_t i = idx % k, j = idx / k;
  R[i + j * ldr] = (i <= j) ? W[i + j * ldw] : 0.0;
}

__global__ __launch_bounds__(256) void iota_kernel(int64_t* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// ---- workspace layouts -----------------------------------------------------
struct SvdWork {
  double *Bt, *J, *Js, *offmax, *sweepmax, *part;
  int* order;
  int64_t ldt, ldj;
  int split;
};

int svd_carve(Arena& a, int64_t m, int64_t n, int64_t k, SvdWork* w) {
  w->ldt = even_up(n);
  w->ldj = even_up(k);
  w->Bt = a.take<double>(static_cast<size_t>(w->ldt) * k);
  w->J = a.take<double>(static_cast<size_t>(w->ldj) * k);
  w->Js = a.take<double>(static_cast<size_t>(w->ldj) * k);
  w->offmax = a.take<double>(static_cast<size_t>(k / 2 + 1));
  w->sweepmax = a.take<double>(1);
  w->order = a.take<int>(static_cast<size_t>(k));
  w->split = choose_split(m, k, k);
  w->part = a.take<double>(partial_doubles(m, k, w->split) + 1);
  return (a.base != nullptr && a.used > a.cap) ? kEWorkspace : kOk;
}

struct QrWork {
  double *W, *vstore, *tau, *Qt, *cval, *part;
  int64_t* cidx;
  int64_t ldw;
  int split;
};

int qr_carve(Arena& a, int64_t m, int64_t n, int64_t k, QrWork* w) {
  w->ldw = even_up(k);
  w->W = a.take<double>(static_cast<size_t>(w->ldw) * n);
  w->vstore = a.take<double>(static_cast<size_t>(w->ldw) * k);
  w->tau = a.take<double>(static_cast<size_t>(k));
  w->Qt = a.take<double>(static_cast<size_t>(w->ldw) * k);
  const size_t ncand = static_cast<size_t>(cdiv(n, kQrCols)) + 1;
  w->cval = a.take<double>(ncand);
  w->cidx = a.take<int64_t>(ncand);
  w->split = choose_split(m, k, k);
  w->part = a.take<double>(partial_doubles(m, k, w->split) + 1);
  return (a.base != nullptr && a.used > a.cap) ? kEWorkspace : kOk;
}

bool post_sizes_ok(int64_t m, int64_t n, int64_t k) {
  return m >= 1 && n >= 1 && k >= 1 && k <= m && k <= kSortMax && n < (int64_t(1) << 31) &&
         m < (int64_t(1) << 31);
}

}  // namespace
}  // namespace qb

using namespace qb;

extern "C" {

size_t qb_svd_workspace_bytes(int64_t m, int64_t n, int64_t k) {
  if (!post_sizes_ok(m, n, k)) return 0;
  Arena a{nullptr, 0, 0};
  SvdWork w;
  svd_carve(a, m, n, k, &w);
  return a.used + 256;
}

int qb_svd(const double* Q, int64_t m, int64_t k, int64_t ldq, const double* B, int64_t n,
           int64_t ldb, double* U, int64_t ldu, double* S, double* V, int64_t ldv,
           int32_t* sweeps, void* workspace, size_t ws_bytes, void* stream) {
  if (!Q || !B || !U || !S || !V || !post_sizes_ok(m, n, k)) return QB_EINVAL;
  if (ldq < m || ldb < k || ldu < m || ldv < n) return QB_EINVAL;
  if (workspace == nullptr) return QB_EWORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EINVAL;
  if (const int dv = device_ready()) return dv;
  SvdWork w;
  Arena arena{static_cast<char*>(workspace), ws_bytes, 0};
  if (svd_carve(arena, m, n, k, &w) != kOk) return QB_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int kk = static_cast<int>(k);
  const int K = kk + (kk & 1);
  hipLaunchKernelGGL(transpose_kernel, dim3(static_cast<unsigned>(cdiv(n, 32)),
                                            static_cast<unsigned>(cdiv(k, 32))),
                     dim3(256), 0, st, B, ldb, w.Bt, w.ldt, k, n);
  hipLaunchKernelGGL(identity_kernel, dim3(static_cast<unsigned>(cdiv(k * k, 256))), dim3(256), 0,
                     st, w.J, w.ldj, kk);
  if (hipGetLastError() != hipSuccess) return QB_EHIP;
  int sw = 0;
  bool converged = (K < 2);
  while (!converged && sw < kMaxSweeps) {
    hipLaunchKernelGGL(zero_kernel1, dim3(static_cast<unsigned>(cdiv(K / 2, 256))), dim3(256), 0,
                       st, w.offmax, static_cast<int64_t>(K / 2));
    for (int r = 0; r < K - 1; ++r)
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(static_cast<unsigned>(K / 2)),
                         dim3(kJacThreads), 0, st, w.Bt, w.ldt, n, w.J, w.ldj, kk, K, r, w.offmax);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, w.offmax,
                       static_cast<int64_t>(K / 2), w.sweepmax);
    if (hipGetLastError() != hipSuccess) return QB_EHIP;
    double hmax = 0.0;
    if (hipMemcpyAsync(&hmax, w.sweepmax, sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QB_EHIP;
    ++sw;
    converged = !(hmax > kJacTol);
  }
  if (sweeps) *sweeps = sw;
  hipLaunchKernelGGL(sigma_sort_kernel, dim3(1), dim3(kSortThreads), 0, st, w.Bt, w.ldt, n, kk, S,
                     w.order);
  hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(k)), dim3(256), 0, st, w.Bt, w.ldt,
                     n, w.J, w.ldj, kk, S, w.order, V, ldv, w.Js);
  if (hipGetLastError() != hipSuccess) return QB_EHIP;
  if (gemm_nn(Q, ldq, w.Js, w.ldj, U, ldu, m, k, k, 1.0, 0.0, w.split, w.part, st)) return QB_EHIP;
  return converged ? QB_OK : QB_NOT_CONVERGED;
}

size_t qb_pivoted_qr_workspace_bytes(int64_t m, int64_t n, int64_t k) {
  if (!post_sizes_ok(m, n, k)) return 0;
  Arena a{nullptr, 0, 0};
  QrWork w;
  qr_carve(a, m, n, k, &w);
  return a.used + 256;
}

int qb_pivoted_qr(const double* Q, int64_t m, int64_t k, int64_t ldq, const double* B, int64_t n,
                  int64_t ldb, double* Qhat, int64_t ldqh, double* R, int64_t ldr, int64_t* perm,
                  void* workspace, size_t ws_bytes, void* stream) {
  if (!Q || !B || !Qhat || !R || !perm || !post_sizes_ok(m, n, k)) return QB_EINVAL;
  if (ldq < m || ldb < k || ldqh < m || ldr < k) return QB_EINVAL;
  if (workspace == nullptr) return QB_EWORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EINVAL;
  if (const int dv = device_ready()) return dv;
  QrWork w;
  Arena arena{static_cast<char*>(workspace), ws_bytes, 0};
  if (qr_carve(arena, m, n, k, &w) != kOk) return QB_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int kk = static_cast<int>(k);
  if (copy_matrix(B, ldb, w.W, w.ldw, k, n, st)) return QB_EHIP;
  hipLaunchKernelGGL(iota_kernel, dim3(static_cast<unsigned>(cdiv(n, 256))), dim3(256), 0, st,
                     perm, n);
  const int steps = static_cast<int>(std::min<int64_t>(k, n));
  hipLaunchKernelGGL(qr_norms_kernel, dim3(static_cast<unsigned>(cdiv(n, kQrCols))),
                     dim3(64 * kQrCols), 0, st, w.W, w.ldw, kk, n, 0, int64_t(0), w.cval, w.cidx);
  for (int j = 0; j < steps; ++j) {
    const int ncand = static_cast<int>(cdiv(n - j, kQrCols));
    hipLaunchKernelGGL(qr_pivot_kernel, dim3(1), dim3(256), 0, st, w.W, w.ldw, kk, j, w.cval,
                       w.cidx, ncand, perm, w.vstore, w.ldw, w.tau);
    const int64_t rest = n - j - 1;
    if (rest > 0)
      hipLaunchKernelGGL(qr_apply_kernel, dim3(static_cast<unsigned>(cdiv(rest, kQrCols))),
                         dim3(64 * kQrCols), 0, st, w.W, w.ldw, kk, n, j, w.vstore, w.ldw, w.tau,
                         w.cval, w.cidx);
    if (hipGetLastError() != hipSuccess) return QB_EHIP;
  }
  hipLaunchKernelGGL(identity_kernel, dim3(static_cast<unsigned>(cdiv(k * k, 256))), dim3(256), 0,
                     st, w.Qt, w.ldw, kk);
  for (int j = steps - 1; j >= 0; --j)
    hipLaunchKernelGGL(qr_accum_kernel, dim3(static_cast<unsigned>(cdiv(k, kQrCols))),
                       dim3(64 * kQrCols), 0, st, w.Qt, w.ldw, kk, j, w.vstore, w.ldw, w.tau);
  hipLaunchKernelGGL(triu_copy_kernel, dim3(static_cast<unsigned>(cdiv(k * n, 256))), dim3(256), 0,
                     st, w.W, w.ldw, R, ldr, kk, n);
  if (hipGetLastError() != hipSuccess) return QB_EHIP;
  if (gemm_nn(Q, ldq, w.Qt, w.ldw, Qhat, ldqh, m, k, k, 1.0, 0.0, w.split, w.part, st))
    return QB_EHIP;
  return QB_OK;
}

}  // extern "C"
