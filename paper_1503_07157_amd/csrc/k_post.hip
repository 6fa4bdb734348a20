// Standard factorisations from A ~ Q B (Section 3.3).
//
// Low-rank SVD (Section 3.3.1).  The SVD of the k x n matrix B comes from
// one-sided (Hestenes) Jacobi on B^T: plane rotations J applied to pairs
// of columns of B^T until all columns are mutually orthogonal, so that
// B^T J = W with orthogonal columns.  Then B = J Sigma (W Sigma^-1)^T:
// the left singular vectors of B are the columns of J, the right ones the
// normalised columns of W, and U = Q J.  Rotating the columns directly
// keeps the high relative accuracy of the small singular values that a
// Gram-matrix route would lose below sqrt(u) sigma_1.  The columns go in
// blocks of two: a round pairs the blocks round-robin (K2 = ceil(k / 2)
// rounded up to even), one workgroup per pair of blocks with their four
// columns in registers, which rotates the four column pairs across the
// blocks (and, in a sweep's first round, the pair inside each block); K2 - 1
// rounds make a sweep, in which every pair of columns meets once.  Columns
// longer than the registers hold (n > 10240) take one pair per workgroup
// and K - 1 rounds of K/2 pairs instead.  Sweeps repeat until every pair is
// orthogonal to a relative 1e-15.  The singular values are
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
#include <cstdint>
#include <type_traits>

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

// ---- two-column blocks -----------------------------------------------------
// The same rotations, ordered by blocks of two columns: block q holds
// columns 2q, 2q + 1 of Bt (a column >= k is absent and stays zero).  In
// round r of a sweep, workgroup i takes the blocks of the round-robin pairing
// of K2 blocks (K2 = ceil(k / 2) rounded up to even) and keeps their four
// columns of Bt in registers while it rotates the four pairs across the two
// blocks, two disjoint pairs at a time, and in round 0 first the pair inside
// each block.  The rotations are recorded in LDS and applied to the four
// (short) columns of J afterwards, in the same order.  Every pair of columns
// still meets once per sweep, every rotation is computed from the columns
// as they are (three dot products in a fixed order), and each column of Bt
// is read and written once per round instead of three times per pair, in
// half as many rounds.

// rotation slot s of a round: pair (jb_p(s), jb_q(s)) of the four columns;
// slots 0, 1 inside the blocks (round 0 only), 2 .. 5 across them
__host__ __device__ constexpr int jb_p(int s) { return s == 0 ? 0 : s == 1 ? 2 : s == 2 ? 0 : s == 3 ? 1 : s == 4 ? 0 : 1; }
__host__ __device__ constexpr int jb_q(int s) { return s == 0 ? 1 : s == 1 ? 3 : s == 2 ? 2 : s == 3 ? 3 : s == 4 ? 3 : 2; }

// slots S and S + 1 (two disjoint pairs): the six dot products, one
// fixed-order workgroup sum, then both rotations on the registers; the
// parameters (c, s), or c = 2 for no rotation, go to rp[slot] (thread 0)
template <int NT, int CAP, int S>
__device__ __forceinline__ void jb_step(double (&x)[4][CAP], double* red, double2* rp,
                                        double& offm, bool& changed) {
  constexpr int P0 = jb_p(S), Q0 = jb_q(S), P1 = jb_p(S + 1), Q1 = jb_q(S + 1);
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < CAP; ++e) {  // absent entries hold zeros
    s[0] = fma(x[P0][e], x[P0][e], s[0]);
    s[1] = fma(x[Q0][e], x[Q0][e], s[1]);
    s[2] = fma(x[P0][e], x[Q0][e], s[2]);
    s[3] = fma(x[P1][e], x[P1][e], s[3]);
    s[4] = fma(x[Q1][e], x[Q1][e], s[4]);
    s[5] = fma(x[P1][e], x[Q1][e], s[5]);
  }
  constexpr int NWV = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[v] += __shfl_xor(s[v], off);
  }
  __syncthreads();  // red is free (the previous step's reads are done)
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < 6; ++v) red[v * NWV + wave] = s[v];
  }
  __syncthreads();
  // thread v < 6 sums value v over the waves in order; then every thread
  // reads the six totals (reading all 6 NWV partials per thread would hold
  // them in registers at once)
  if (threadIdx.x < 6) {
    const int v = threadIdx.x;
    double t = red[v * NWV];
    for (int w = 1; w < NWV; ++w) t += red[v * NWV + w];
    red[6 * NWV + v] = t;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 6; ++v) s[v] = red[6 * NWV + v];
  auto rot = [&](auto pc, auto qc, int slot, double alpha, double beta, double gamma) {
    constexpr int P = decltype(pc)::value, Q = decltype(qc)::value;
    double off = 0.0;
    if (alpha > 0.0 && beta > 0.0) off = fabs(gamma) / (sqrt(alpha) * sqrt(beta));
    offm = fmax(offm, off);
    if (!(off > kJacTol)) {  // also every pair with an absent column
      if (threadIdx.x == 0) rp[slot] = make_double2(2.0, 0.0);
      return;
    }
    const double zeta = (beta - alpha) / (2.0 * gamma);
    const double az = fabs(zeta);
    const double tt = (az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az)));
    const double t = zeta >= 0.0 ? tt : -tt;
    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
    for (int e = 0; e < CAP; ++e) {
      const double xa = x[P][e], yb = x[Q][e];
      x[P][e] = c * xa - sn * yb;
      x[Q][e] = sn * xa + c * yb;
    }
    if (threadIdx.x == 0) rp[slot] = make_double2(c, sn);
    changed = true;
  };
  rot(std::integral_constant<int, P0>{}, std::integral_constant<int, Q0>{}, S, s[0], s[1], s[2]);
  rot(std::integral_constant<int, P1>{}, std::integral_constant<int, Q1>{}, S + 1, s[3], s[4],
      s[5]);
}

template <int NT, int CAP>
__global__ __launch_bounds__(NT) void jacobi_block_round_kernel(
    double* __restrict__ Bt, int64_t ldt, int n, double* __restrict__ J, int64_t ldj, int k,
    int K2, int r, double* __restrict__ offmax) {
  __shared__ double red[6 * (NT / 64) + 6];
  __shared__ double2 rp[6];
  const int i = blockIdx.x, t = threadIdx.x;
  int ba = rr_index(i, r, K2), bb = rr_index(K2 - 1 - i, r, K2);
  if (ba > bb) { const int u = ba; ba = bb; bb = u; }
  const int nb = (k + 1) / 2;  // blocks holding a column
  if (ba >= nb) return;        // both blocks are padding
  const bool hasb = bb < nb;
  const int col[4] = {2 * ba, 2 * ba + 1, 2 * bb, 2 * bb + 1};
  const bool here[4] = {true, col[1] < k, hasb, hasb && col[3] < k};
  double x[4][CAP];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* src = Bt + static_cast<int64_t>(col[q]) * ldt;
#pragma unroll
    for (int e = 0; e < CAP; ++e) {
      const int idx = t + NT * e;
      x[q][e] = (here[q] && idx < n) ? src[idx] : 0.0;
    }
  }
  double offm = 0.0;
  bool changed = false;
  if (r == 0) jb_step<NT, CAP, 0>(x, red, rp, offm, changed);
  if (hasb) {
    jb_step<NT, CAP, 2>(x, red, rp, offm, changed);
    jb_step<NT, CAP, 4>(x, red, rp, offm, changed);
  }
  if (t == 0) offmax[i] = fmax(offmax[i], offm);
  if (!changed) return;  // uniform: every thread took the same decisions
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!here[q]) continue;
    double* dst = Bt + static_cast<int64_t>(col[q]) * ldt;
#pragma unroll
    for (int e = 0; e < CAP; ++e) {
      const int idx = t + NT * e;
      if (idx < n) dst[idx] = x[q][e];
    }
  }
  __syncthreads();  // rp written by thread 0
  // J: the recorded rotations in order, on the entries each thread owns;
  // the columns of absent indices are never rotated, so never touched
  const int s0 = r == 0 ? 0 : 2, s1 = hasb ? 6 : 2;
  for (int q = t; q < k; q += NT) {
    double jx[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) jx[c] = here[c] ? J[q + static_cast<int64_t>(col[c]) * ldj] : 0.0;
    bool hit[4] = {false, false, false, false};
#pragma unroll
    for (int sl = 0; sl < 6; ++sl) {
      if (sl < s0 || sl >= s1) continue;
      const double2 cs = rp[sl];
      if (cs.x > 1.5) continue;
      const int P = jb_p(sl), Q = jb_q(sl);
      const double xa = jx[P], yb = jx[Q];
      jx[P] = cs.x * xa - cs.y * yb;
      jx[Q] = cs.y * xa + cs.x * yb;
      hit[P] = hit[Q] = true;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (hit[c]) J[q + static_cast<int64_t>(col[c]) * ldj] = jx[c];
  }
}

// one round of the blocked form, the columns of n held in CAP registers
// per thread (512 threads, or 1024 for the longest columns: four columns
// of 20 entries per thread spilled); jb_fits: some instance holds them
bool jb_fits(int64_t n) { return n <= 10240; }
void jb_launch(int n, dim3 g, hipStream_t st, double* Bt, int64_t ldt, double* J, int64_t ldj,
               int k, int K2, int r, double* offmax) {
  auto go = [&](auto ntc, auto capc) {
    constexpr int NT = decltype(ntc)::value, CAP = decltype(capc)::value;
    hipLaunchKernelGGL((jacobi_block_round_kernel<NT, CAP>), g, dim3(NT), 0, st, Bt, ldt, n, J,
                       ldj, k, K2, r, offmax);
  };
  using I = std::integral_constant<int, 512>;
  if (n <= 512 * 4) go(I{}, std::integral_constant<int, 4>{});
  else if (n <= 512 * 8) go(I{}, std::integral_constant<int, 8>{});
  else if (n <= 512 * 12) go(I{}, std::integral_constant<int, 12>{});
  else go(std::integral_constant<int, 1024>{}, std::integral_constant<int, 10>{});
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
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  __shared__ int64_t piv;
  // argmax over the candidates, ties to the smaller index: each thread scans
  // a strided share, then a tree in LDS (the winner is unique, so the order
  // of the comparisons does not change it)
  {
    double v = -2.0;
    int64_t id = INT64_MAX;
    for (int c = threadIdx.x; c < ncand; c += 256) {
      const double cv = cval[c];
      const int64_t ci = cidx[c];
      if (cv > v || (cv == v && ci < id)) { v = cv; id = ci; }
    }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = id;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (static_cast<int>(threadIdx.x) < h) {
        const double ov = bv[threadIdx.x + h];
        const int64_t oi = bi[threadIdx.x + h];
        if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
          bv[threadIdx.x] = ov;
          bi[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) piv = bi[0];
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
template <int KC>
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
    // the column's rows j.. (KC per lane) are loaded once and kept in
    // registers for the dot product, the update and the next norm; sums in
    // the same per-lane order as a strided loop
    double* c = W + col * ldw;
    double cr[KC], vr[KC];
#pragma unroll
    for (int e = 0; e < KC; ++e) {
      const int t = j + lane + 64 * e;
      cr[e] = t < k ? c[t] : 0.0;
      vr[e] = t < k ? v[t] : 0.0;
    }
    double d = 0.0;
#pragma unroll
    for (int e = 0; e < KC; ++e)
      if (j + lane + 64 * e < k) d = fma(vr[e], cr[e], d);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
    const double f = tj * d;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < KC; ++e) {
      const int t = j + lane + 64 * e;
      if (t < k) {
        const double u = cr[e] - f * vr[e];
        c[t] = u;
        if (t > j) acc = fma(u, u, acc);
      }
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

// qr_apply_kernel with registers for rows = k - j rows per column (k <= 4096)
void qr_apply(int rows, dim3 g, hipStream_t st, double* W, int64_t ldw, int k, int64_t n, int j,
              const double* vstore, int64_t ldv, const double* tau, double* cval, int64_t* cidx) {
  auto go = [&](auto kc) {
    constexpr int KC = decltype(kc)::value;
    hipLaunchKernelGGL((qr_apply_kernel<KC>), g, dim3(64 * kQrCols), 0, st, W, ldw, k, n, j,
                       vstore, ldv, tau, cval, cidx);
  };
  const int need = (rows + 63) / 64;
  if (need <= 1) go(std::integral_constant<int, 1>{});
  else if (need <= 2) go(std::integral_constant<int, 2>{});
  else if (need <= 4) go(std::integral_constant<int, 4>{});
  else if (need <= 8) go(std::integral_constant<int, 8>{});
  else if (need <= 16) go(std::integral_constant<int, 16>{});
  else if (need <= 24) go(std::integral_constant<int, 24>{});
  else if (need <= 32) go(std::integral_constant<int, 32>{});
  else if (need <= 48) go(std::integral_constant<int, 48>{});
  else go(std::integral_constant<int, 64>{});
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
  // two-column blocks when four columns of Bt and of J fit in registers,
  // else one pair per workgroup
  const bool blocked = jb_fits(n);
  const int K2 = static_cast<int>(even_up((k + 1) / 2));
  const int slots = blocked ? K2 / 2 : K / 2;
  while (!converged && sw < kMaxSweeps) {
    hipLaunchKernelGGL(zero_kernel1, dim3(static_cast<unsigned>(cdiv(slots, 256))), dim3(256), 0,
                       st, w.offmax, static_cast<int64_t>(slots));
    if (blocked) {
      for (int r = 0; r < K2 - 1; ++r)
        jb_launch(static_cast<int>(n), dim3(static_cast<unsigned>(K2 / 2)), st, w.Bt, w.ldt, w.J,
                  w.ldj, kk, K2, r, w.offmax);
    } else {
      for (int r = 0; r < K - 1; ++r)
        hipLaunchKernelGGL(jacobi_round_kernel, dim3(static_cast<unsigned>(K / 2)),
                           dim3(kJacThreads), 0, st, w.Bt, w.ldt, n, w.J, w.ldj, kk, K, r,
                           w.offmax);
    }
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, w.offmax,
                       static_cast<int64_t>(slots), w.sweepmax);
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
      qr_apply(kk - j, dim3(static_cast<unsigned>(cdiv(rest, kQrCols))), st, w.W, w.ldw, kk, n, j,
               w.vstore, w.ldw, w.tau, w.cval, w.cidx);
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
