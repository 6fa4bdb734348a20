// Gradient of the fixed-sketch QB map A -> (Q, B).
//
// With the Gaussian sketch (seed), the block width b, the number of blocks s
// and the number of power iterations P held fixed, the blocked scheme of
// Figures 4 and 6 is a smooth function of A wherever every orthonormalisation
// sees a full-column-rank matrix (orth(X) is then the Q factor of the thin QR
// of X with positive diagonal, Section 2.4):
//
//   R_0 = A;  for i = 1 .. s:
//     Q^0 = orth(R_{i-1} Omega_i)
//     p = 1 .. P:  Z^p = orth(R_{i-1}^T Q^{p-1});  Q^p = orth(R_{i-1} Z^p)
//     i > 1:  C = Qbar^T Q^P,  Q_i = orth(Q^P - Qbar C)      (Section 4.3)
//     i = 1:  Q_i = Q^P
//     B_i = Q_i^T R_{i-1};  R_i = R_{i-1} - Q_i B_i
//
// qb_adjoint returns dA = J^T (dQ, dB), the vector-Jacobian product, by
// running the blocks in reverse.  Nothing of the forward is stored but Q and
// B: each block's samples Y = R_{i-1} Omega_i and the power-iteration
// intermediates are recomputed from A, Q and B, with R_{i-1} X = A X -
// Qbar (Bbar X) and R_{i-1}^T X = A^T X - Bbar^T (Qbar^T X), so no m x n
// matrix besides A and dA is held.  The adjoint of X -> Q (thin QR, R not
// used downstream) is
//
//   Xbar = (Qbar_in - Q S) R^{-T},  S = triu(N) + tril(N^T, -1),  N = Q^T Qbar_in,
//
// with R^{-1} = T1^{-1} T2^{-1} from the two Cholesky QR passes.  The
// contributions of one block to dA (from B_i, the sketch and each power
// product) are gathered as one rank-(2 + 2P) b update.
#include <algorithm>
#include <vector>

#include "../../include/qb.h"
#include "qb_internal.hpp"

namespace qb {
namespace {

constexpr int kAdjMaxPower = 8;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t even_up(int64_t v) { return (v + 1) & ~int64_t(1); }

// Y (N x M, ldy) = X^T for X (M x N, ldx); 32 x 32 tiles through LDS
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ Y, int64_t ldy,
                                                        int64_t M, int64_t N) {
  __shared__ double t[32][33];
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 32, j0 = static_cast<int64_t>(blockIdx.y) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + tx, j = j0 + r;
    if (i < M && j < N) t[r][tx] = X[i + j * ldx];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + tx, i = i0 + r;
    if (j < N && i < M) Y[j + i * ldy] = t[tx][r];
  }
}

// Y += alpha X (M x N)
__global__ __launch_bounds__(256) void axpy_kernel(double alpha, const double* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ Y, int64_t ldy,
                                                   int64_t M, int64_t N) {
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y)
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < M;
         i += static_cast<int64_t>(gridDim.x) * 256)
      Y[i + j * ldy] += alpha * X[i + j * ldx];
}

// S = triu(N) + tril(N^T, -1), w x w, ld w
__global__ __launch_bounds__(256) void sym_upper_kernel(const double* __restrict__ Nm, int w,
                                                        double* __restrict__ S) {
  const int64_t total = static_cast<int64_t>(w) * w;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t i = e % w, j = e / w;
    S[e] = i <= j ? Nm[i + j * w] : Nm[j + i * w];
  }
}

int transpose(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t M, int64_t N,
              hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  hipLaunchKernelGGL(transpose_kernel, dim3(static_cast<unsigned>(cdiv(M, 32)),
                                            static_cast<unsigned>(cdiv(N, 32))),
                     dim3(256), 0, s, X, ldx, Y, ldy, M, N);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int axpy(double alpha, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t M, int64_t N,
         hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  const dim3 grid(static_cast<unsigned>(std::min<int64_t>(cdiv(M, 256), 64)),
                  static_cast<unsigned>(std::min<int64_t>(N, 4096)));
  hipLaunchKernelGGL(axpy_kernel, grid, dim3(256), 0, s, alpha, X, ldx, Y, ldy, M, N);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

struct Dims {
  int64_t m, n, lda, ldq, ldb;
  int w, blocks, P;
  int64_t ldm, ldn, kmax, Kr;
};

struct AdjWork {
  double *dQw, *Om, *Y, *Qp, *Ri, *Z, *Rz, *tm, *tn, *C, *Xr, *Qr, *Rr, *Tw, *Bt, *GBt, *Tk, *T3,
      *Xb, *H, *Ct, *Ht, *Gp, *Zb, *Wb, *Nw, *Sw, *RiT, *t1, *tq, *Lf, *Rf, *part;
  int* dropped;
  OrthWork ow;
};

// the products of the backward, for sizing the split-K buffer
template <class F>
void each_product(const Dims& d, F f) {
  const int64_t m = d.m, n = d.n, w = d.w;
  for (int i = 0; i < d.blocks; ++i) {
    const int64_t k = static_cast<int64_t>(i) * w;
    f(m, w, n);            // A X, R-bar B_i^T, A dB_i^T
    f(n, w, m);            // A^T X
    f(w, n, m);            // Q_i^T R-bar
    f(w, w, std::max(m, n));  // Q^T G in the orth adjoint
    f(m, w, w);            // (G - Q S) R^{-T}, Q S, on m rows
    f(n, w, w);            // the same on n rows (power iterations)
    f(m, n, d.Kr);         // rank update of dA
    if (k > 0) {
      f(k, w, n);          // Bbar X
      f(m, w, k);          // Qbar (.)
      f(k, w, m);          // Qbar^T X
      f(n, w, k);          // Bbar^T (.)
      f(m, k, w);          // dQbar updates
    }
  }
}

int carve_adj(Arena& a, const Dims& d, AdjWork* W) {
  const int64_t w = d.w, P = d.P, ldm = d.ldm, ldn = d.ldn, kmax = std::max<int64_t>(d.kmax, 1);
  const int64_t ldmn = std::max(ldm, ldn);
  W->dQw = a.take<double>(static_cast<size_t>(ldm) * d.blocks * w);
  W->Om = a.take<double>(static_cast<size_t>(ldn) * w);
  W->Y = a.take<double>(static_cast<size_t>(ldm) * w);
  W->Qp = a.take<double>(static_cast<size_t>(ldm) * w * (P + 1));
  W->Ri = a.take<double>(static_cast<size_t>(w) * w * (P + 1));
  W->Z = a.take<double>(static_cast<size_t>(ldn) * w * std::max<int64_t>(P, 1));
  W->Rz = a.take<double>(static_cast<size_t>(w) * w * std::max<int64_t>(P, 1));
  W->tm = a.take<double>(static_cast<size_t>(ldm) * w);
  W->tn = a.take<double>(static_cast<size_t>(ldn) * w);
  W->C = a.take<double>(static_cast<size_t>(kmax) * w);
  W->Xr = a.take<double>(static_cast<size_t>(ldm) * w);
  W->Qr = a.take<double>(static_cast<size_t>(ldm) * w);
  W->Rr = a.take<double>(static_cast<size_t>(w) * w);
  W->Tw = a.take<double>(static_cast<size_t>(w) * d.n);
  W->Bt = a.take<double>(static_cast<size_t>(ldn) * w);
  W->GBt = a.take<double>(static_cast<size_t>(ldn) * w);
  W->Tk = a.take<double>(static_cast<size_t>(kmax) * w);
  W->T3 = a.take<double>(static_cast<size_t>(ldn) * w);
  W->Xb = a.take<double>(static_cast<size_t>(ldm) * w);
  W->H = a.take<double>(static_cast<size_t>(kmax) * w);
  W->Ct = a.take<double>(static_cast<size_t>(w) * kmax);
  W->Ht = a.take<double>(static_cast<size_t>(w) * kmax);
  W->Gp = a.take<double>(static_cast<size_t>(ldm) * w);
  W->Zb = a.take<double>(static_cast<size_t>(ldn) * w);
  W->Wb = a.take<double>(static_cast<size_t>(ldn) * w);
  W->Nw = a.take<double>(static_cast<size_t>(w) * w);
  W->Sw = a.take<double>(static_cast<size_t>(w) * w);
  W->RiT = a.take<double>(static_cast<size_t>(w) * w);
  W->t1 = a.take<double>(static_cast<size_t>(w) * w);
  W->tq = a.take<double>(static_cast<size_t>(ldmn) * w);
  W->Lf = a.take<double>(static_cast<size_t>(ldm) * d.Kr);
  W->Rf = a.take<double>(static_cast<size_t>(d.Kr) * d.n);
  size_t part = 1;
  each_product(d, [&](int64_t M, int64_t N, int64_t K) {
    part = std::max(part, partial_doubles(M, N, choose_split(M, N, K)));
    part = std::max(part, partial_doubles(M, N, choose_split(M, N, K, 2, true)));
  });
  W->part = a.take<double>(part);
  W->dropped = a.take<int>(2);
  if (orth_carve(a, std::max(d.m, d.n), d.w, &W->ow) != kOk) return kEWorkspace;
  return (a.base != nullptr && a.used > a.cap) ? kEWorkspace : kOk;
}

// products with the shared split-K buffer
struct Mm {
  double* part;
  hipStream_t s;
  int nn(const double* X, int64_t ldx, const double* Wm, int64_t ldw, double* Y, int64_t ldy,
         int64_t M, int64_t N, int64_t K, double alpha, double beta) const {
    return gemm_nn(X, ldx, Wm, ldw, Y, ldy, M, N, K, alpha, beta, choose_split(M, N, K, 2, true),
                   part, s);
  }
  int tn(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C, int64_t ldc,
         int64_t P, int64_t N, int64_t K) const {
    return gemm_tn(Qm, ldq, X, ldx, C, ldc, P, N, K, false, choose_split(P, N, K), part, nullptr,
                   nullptr, s);
  }
};

}  // namespace
}  // namespace qb

using namespace qb;

namespace {

bool adj_dims(int64_t m, int64_t n, int64_t lda, int32_t b, int32_t blocks, int32_t power_iters,
              int64_t ldq, int64_t ldb, Dims* d) {
  if (m < 1 || n < 1 || b < 1 || b > kMaxPanel || blocks < 1 || power_iters < 0 ||
      power_iters > kAdjMaxPower)
    return false;
  const int64_t ktot = static_cast<int64_t>(b) * blocks;
  if (ktot > std::min(m, n)) return false;
  if (lda < m || ldq < m || ldb < ktot) return false;
  const int64_t lim = int64_t(1) << 24;
  if (lda >= lim || ldq >= lim || ldb >= lim || m >= lim || n >= lim) return false;
  d->m = m;
  d->n = n;
  d->lda = lda;
  d->ldq = ldq;
  d->ldb = ldb;
  d->w = b;
  d->blocks = blocks;
  d->P = power_iters;
  d->ldm = even_up(m);
  d->ldn = even_up(n);
  d->kmax = static_cast<int64_t>(blocks - 1) * b;
  d->Kr = static_cast<int64_t>(2 + 2 * power_iters) * b;
  return true;
}

}  // namespace

extern "C" {

size_t qb_adjoint_workspace_bytes(int64_t m, int64_t n, int32_t b, int32_t blocks,
                                  int32_t power_iters) {
  Dims d;
  if (!adj_dims(m, n, m, b, blocks, power_iters, m, static_cast<int64_t>(b) * std::max(blocks, 1),
                &d))
    return 0;
  Arena a{nullptr, 0, 0};
  AdjWork W;
  carve_adj(a, d, &W);
  return a.used + 256;
}

int qb_adjoint(const double* A, int64_t m, int64_t n, int64_t lda, int32_t b, int32_t blocks,
               int32_t power_iters, uint64_t seed, const double* Q, int64_t ldq, const double* B,
               int64_t ldb, const double* dQ, int64_t lddq, const double* dB, int64_t lddb,
               double* dA, int64_t ldda, void* workspace, size_t ws_bytes, void* stream) {
  Range rcall("qb_adjoint");
  Dims d;
  if (!A || !Q || !B || !dA) return QB_EINVAL;
  if (!adj_dims(m, n, lda, b, blocks, power_iters, ldq, ldb, &d)) return QB_EINVAL;
  const int64_t ktot = static_cast<int64_t>(b) * blocks;
  if (ldda < m || ldda >= (int64_t(1) << 24)) return QB_EINVAL;
  if (dQ && (lddq < m || lddq >= (int64_t(1) << 24))) return QB_EINVAL;
  if (dB && (lddb < ktot || lddb >= (int64_t(1) << 24))) return QB_EINVAL;
  if (!workspace) return QB_EWORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EINVAL;
  if (const int dv = device_ready()) return dv;
  Arena arena{static_cast<char*>(workspace), ws_bytes, 0};
  AdjWork W;
  if (carve_adj(arena, d, &W) != kOk) return QB_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Mm mm{W.part, st};
  const int w = d.w, P = d.P;
  const int64_t ldm = d.ldm, ldn = d.ldn, Kr = d.Kr;
  const int64_t ldqw = ldm;
  const int64_t lkm = std::max<int64_t>(d.kmax, 1);

  auto run = [&]() -> int {
    if (zero_matrix(dA, ldda, m, n, st)) return 1;
    if (dQ) {
      if (copy_matrix(dQ, lddq, W.dQw, ldqw, m, ktot, st)) return 1;
    } else if (zero_matrix(W.dQw, ldqw, m, ktot, st)) {
      return 1;
    }
    if (zero_matrix(reinterpret_cast<double*>(W.dropped), 1, 1, 1, st)) return 1;  // both ints
    for (int i = blocks - 1; i >= 0; --i) {
      const int64_t k = static_cast<int64_t>(i) * w;
      const double* Qi = Q + k * ldq;
      const double* Bi = B + k;
      double* GQ = W.dQw + k * ldqw;
      // R_{i-1} X (X: n x w) and R_{i-1}^T X (X: m x w)
      auto Rprod = [&](const double* X, int64_t ldx, double* out, int64_t ldo) -> int {
        if (mm.nn(A, d.lda, X, ldx, out, ldo, m, w, n, 1.0, 0.0)) return 1;
        if (k == 0) return 0;
        if (mm.nn(B, d.ldb, X, ldx, W.Tk, lkm, k, w, n, 1.0, 0.0)) return 1;
        return mm.nn(Q, d.ldq, W.Tk, lkm, out, ldo, m, w, k, -1.0, 1.0);
      };
      auto RTprod = [&](const double* X, int64_t ldx, double* out, int64_t ldo) -> int {
        if (mm.tn(A, d.lda, X, ldx, out, ldo, n, w, m)) return 1;
        if (k == 0) return 0;
        if (mm.tn(Q, d.ldq, X, ldx, W.Tk, lkm, k, w, m)) return 1;
        if (mm.tn(B, d.ldb, W.Tk, lkm, W.T3, ldn, n, w, k)) return 1;
        return axpy(-1.0, W.T3, ldn, out, ldo, n, w, st);
      };
      auto orth = [&](const double* X, int64_t ldx, int64_t rows, double* Qo, int64_t ldo,
                      double* rinv) -> int {
        return orth_cholqr2_rinv(X, ldx, Qo, ldo, rows, w, W.ow, W.t1, rinv, W.dropped, st);
      };
      // Xbar = (G - Q S) R^{-T}, S from N = Q^T G
      auto qr_adj = [&](const double* Qm, int64_t ldqm, const double* rinv, const double* G,
                        int64_t ldg, int64_t rows, double* out, int64_t ldo) -> int {
        if (mm.tn(Qm, ldqm, G, ldg, W.Nw, w, w, w, rows)) return 1;
        hipLaunchKernelGGL(sym_upper_kernel, dim3(static_cast<unsigned>(cdiv(int64_t(w) * w, 256))),
                           dim3(256), 0, st, W.Nw, w, W.Sw);
        if (hipGetLastError() != hipSuccess) return 1;
        if (copy_matrix(G, ldg, W.tq, std::max(ldm, ldn), rows, w, st)) return 1;
        if (mm.nn(Qm, ldqm, W.Sw, w, W.tq, std::max(ldm, ldn), rows, w, w, -1.0, 1.0)) return 1;
        if (transpose(rinv, w, W.RiT, w, w, w, st)) return 1;
        return mm.nn(W.tq, std::max(ldm, ldn), W.RiT, w, out, ldo, rows, w, w, 1.0, 0.0);
      };
      double* Qp = W.Qp;
      auto QpAt = [&](int p) { return Qp + static_cast<int64_t>(p) * ldm * w; };
      auto RiAt = [&](int p) { return W.Ri + static_cast<int64_t>(p) * w * w; };
      auto ZAt = [&](int p) { return W.Z + static_cast<int64_t>(p - 1) * ldn * w; };
      auto RzAt = [&](int p) { return W.Rz + static_cast<int64_t>(p - 1) * w * w; };
      double* Lb = W.Lf;  // left factors of the rank update, m x Kr (ld ldm)
      double* Rb = W.Rf;  // right factors, Kr x n (ld Kr)
      auto Lblk = [&](int j) { return Lb + static_cast<int64_t>(j) * w * ldm; };
      auto Rblk = [&](int j) { return Rb + static_cast<int64_t>(j) * w; };

      // ---- recompute the forward of block i ----------------------------
      if (launch_sketch(seed, n, k, w, W.Om, ldn, st)) return 1;
      if (Rprod(W.Om, ldn, W.Y, ldm)) return 1;
      if (orth(W.Y, ldm, m, QpAt(0), ldm, RiAt(0))) return 1;
      for (int p = 1; p <= P; ++p) {
        if (RTprod(QpAt(p - 1), ldm, W.tn, ldn)) return 1;
        if (orth(W.tn, ldn, n, ZAt(p), ldn, RzAt(p))) return 1;
        if (Rprod(ZAt(p), ldn, W.tm, ldm)) return 1;
        if (orth(W.tm, ldm, m, QpAt(p), ldm, RiAt(p))) return 1;
      }
      const double* Qprime = QpAt(P);
      if (k > 0) {
        if (mm.tn(Q, d.ldq, Qprime, ldm, W.C, lkm, k, w, m)) return 1;
        if (copy_matrix(Qprime, ldm, W.Xr, ldm, m, w, st)) return 1;
        if (mm.nn(Q, d.ldq, W.C, lkm, W.Xr, ldm, m, w, k, -1.0, 1.0)) return 1;
        if (orth(W.Xr, ldm, m, W.Qr, ldm, W.Rr)) return 1;
      }

      // ---- reverse: R_i = R_{i-1} - Q_i B_i and B_i = Q_i^T R_{i-1} ----
      double* GB = Rblk(0);  // w x n, ld Kr
      if (dB) {
        if (copy_matrix(dB + k, lddb, GB, Kr, w, n, st)) return 1;
      } else if (zero_matrix(GB, Kr, w, n, st)) {
        return 1;
      }
      if (transpose(Bi, d.ldb, W.Bt, ldn, w, n, st)) return 1;
      if (mm.nn(dA, ldda, W.Bt, ldn, GQ, ldqw, m, w, n, -1.0, 1.0)) return 1;
      if (mm.tn(Qi, d.ldq, dA, ldda, W.Tw, w, w, n, m)) return 1;
      if (axpy(-1.0, W.Tw, w, GB, Kr, w, n, st)) return 1;
      if (transpose(GB, Kr, W.GBt, ldn, w, n, st)) return 1;
      if (mm.nn(A, d.lda, W.GBt, ldn, GQ, ldqw, m, w, n, 1.0, 1.0)) return 1;
      if (k > 0) {
        if (mm.nn(B, d.ldb, W.GBt, ldn, W.Tk, lkm, k, w, n, 1.0, 0.0)) return 1;
        if (mm.nn(Q, d.ldq, W.Tk, lkm, GQ, ldqw, m, w, k, -1.0, 1.0)) return 1;
      }
      if (copy_matrix(Qi, d.ldq, Lblk(0), ldm, m, w, st)) return 1;

      // ---- re-projection and its orth ------------------------------------
      if (k > 0) {
        if (qr_adj(W.Qr, ldm, W.Rr, GQ, ldqw, m, W.Xb, ldm)) return 1;
        if (mm.tn(Q, d.ldq, W.Xb, ldm, W.H, lkm, k, w, m)) return 1;
        if (copy_matrix(W.Xb, ldm, W.Gp, ldm, m, w, st)) return 1;
        if (mm.nn(Q, d.ldq, W.H, lkm, W.Gp, ldm, m, w, k, -1.0, 1.0)) return 1;
        if (transpose(W.C, lkm, W.Ct, w, k, w, st)) return 1;
        if (transpose(W.H, lkm, W.Ht, w, k, w, st)) return 1;
        if (mm.nn(W.Xb, ldm, W.Ct, w, W.dQw, ldqw, m, k, w, -1.0, 1.0)) return 1;
        if (mm.nn(Qprime, ldm, W.Ht, w, W.dQw, ldqw, m, k, w, -1.0, 1.0)) return 1;
      } else if (copy_matrix(GQ, ldqw, W.Gp, ldm, m, w, st)) {
        return 1;
      }

      // ---- power iterations, last first ----------------------------------
      for (int p = P; p >= 1; --p) {
        double* Vb = Lblk(2 * p);
        if (qr_adj(QpAt(p), ldm, RiAt(p), W.Gp, ldm, m, Vb, ldm)) return 1;
        if (transpose(ZAt(p), ldn, Rblk(2 * p), Kr, n, w, st)) return 1;
        if (RTprod(Vb, ldm, W.Zb, ldn)) return 1;
        if (qr_adj(ZAt(p), ldn, RzAt(p), W.Zb, ldn, n, W.Wb, ldn)) return 1;
        if (transpose(W.Wb, ldn, Rblk(2 * p + 1), Kr, n, w, st)) return 1;
        if (copy_matrix(QpAt(p - 1), ldm, Lblk(2 * p + 1), ldm, m, w, st)) return 1;
        if (Rprod(W.Wb, ldn, W.Gp, ldm)) return 1;
      }

      // ---- the sample Y = R_{i-1} Omega_i --------------------------------
      if (qr_adj(QpAt(0), ldm, RiAt(0), W.Gp, ldm, m, Lblk(1), ldm)) return 1;
      if (transpose(W.Om, ldn, Rblk(1), Kr, n, w, st)) return 1;

      // ---- dA += [Q_i, Ybar, Vbar_p, Q^{p-1}] [dB_i; Omega^T; Z_p^T; Wbar_p^T]
      if (mm.nn(Lb, ldm, Rb, Kr, dA, ldda, m, n, Kr, 1.0, 1.0)) return 1;
    }
    return 0;
  };
  if (run()) return QB_EHIP;
  int dropped = 0;
  if (hipMemcpyAsync(&dropped, W.dropped, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QB_EHIP;
  return dropped ? QB_RANK_EXHAUSTED : QB_OK;
}

}  // extern "C"
