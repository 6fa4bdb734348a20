// C ABI and host driver of the blocked randomized QB factorisation
// (randQB_b, Figure 4; randQB_pb, Figure 6).  All device work is issued on
// the caller's stream from carved caller workspace; the only host
// synchronisation is one small device-to-host read per block for the
// stopping rule (Section 4.2), plus one at the start for ||A||_F.
//
// Per block (A is the residual, overwritten as in eq. (def3)):
//   Omega_i = sketch columns [k, k+w)                          Fig. 4 (2)
//   Y = A Omega_i;  Q_i = orth(Y)                               Fig. 4 (3)
//   P times: Z = orth(A^T Q_i);  Q_i = orth(A Z)                Fig. 6 (4)-(7)
//   Q_i = orth(Q_i - Qbar (Qbar^T Q_i))                         Fig. 4 (3')
//   B_i = Q_i^T A;  A = A - Q_i B_i  (+ ||A||_F^2)              Fig. 4 (4),(5)
//   stop when the residual norm is at most eps                  Fig. 4 (6)
// The stopping quantity is tracked as E_i = ||A||^2 - sum_j ||B_j||^2
// (Proposition 4.1 (a),(b) and Pythagoras) and, inside a band of
// half-width 1e-13 ||A||^2 around eps^2 where E_i cannot resolve the
// threshold, decided by the directly computed D_i = ||A^(i)||_F^2.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <optional>

#include "../../include/qb.h"
#include "qb_internal.hpp"

namespace qb {
int sum_partials_ex(const double* part, int count, const int* flags, double* out, int* out_flag,
                    hipStream_t s);

namespace {

constexpr double kDeltaRel = 1e-13;               // hybrid band, relative to ||A||_F^2
constexpr double kDeltaRelF32 = 1e-6;             // same, B_i = Q_i^T A in f32
constexpr double kDeltaRelBf16x3 = 1e-4;          // same, B_i in bf16x3
constexpr double kFloorRel = 0x1p-46;             // rounding floor of the residual, rel. ||A||_F

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t even_up(int64_t x) { return (x + 1) & ~int64_t(1); }

// ---- double-double helpers (host) ------------------------------------------
struct DD { double hi, lo; };
inline DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
inline DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  const double e = s.lo + a.lo + b.lo;
  return two_sum(s.hi, e);
}
inline double dd_val(DD a) { return a.hi + a.lo; }

// ---- workspace plan ----------------------------------------------------------
struct Work {
  double* R = nullptr;
  int64_t ldr = 0;
  int64_t ldm = 0;        // leading dimension of m-row panels
  double* omega = nullptr;  // n x b
  double* Y = nullptr;      // m x b
  double* Qi = nullptr;     // m x b
  double* Z = nullptr;      // n x b
  double* C = nullptr;      // kcap x b
  int64_t ldc = 1;
  double* part = nullptr;   // split-K partials
  double* sq1 = nullptr;    // per-workgroup sums of squares (B_i, ||A||)
  double* sq2 = nullptr;    // per-workgroup sums of squares (residual)
  int* flags = nullptr;     // per-workgroup non-finite flags
  double* scal = nullptr;   // [0,1] D_i (hi, lo); [2,3] ||B_i||^2; [4,5] ||A||^2
  int* iscal = nullptr;     // [0] non-finite flag
  int8_t* omq = nullptr;    // int8 sketch of the exact-range sample (QB_SAMPLE_INT8X8)
  OrthWork ow{};
};

size_t max_partials(int64_t m, int64_t n, int b, int64_t kcap, bool exact) {
  size_t best = exact ? sample_i8_partials(m, b, n) : 1;
  auto upd = [&](int64_t rows, int64_t cols, int64_t K) {
    for (bool nn : {false, true}) {
      const int s = choose_split(rows, cols, K, 2, nn);
      const size_t v = partial_doubles(rows, cols, s);
      if (v > best) best = v;
    }
  };
  upd(m, b, n);                // Y = A Omega, Y = A Z
  upd(b, n, m);                // B_i = Q^T A, (A^T Q)^T
  for (int lp : {1, 2}) {      // their low-precision forms (packed panel + partials)
    best = std::max(best, lowp_scratch_doubles(lp, true, m, b, n));
    best = std::max(best, lowp_scratch_doubles(lp, false, b, n, m));
  }
  for (int64_t k = 1; k <= kcap; ++k) {
    upd(b, k, m);              // Q_i^T Qbar (split is not monotone in k)
    upd(m, b, k);              // Qbar C
  }
  return best;
}

size_t max_sq(int64_t m, int64_t n, int b) {
  size_t v = downdate_partials(m, n);
  v = std::max(v, sumsq_partials_count(m, n));
  v = std::max(v, static_cast<size_t>(cdiv(static_cast<int64_t>(b) * n, 256)));
  v = std::max(v, static_cast<size_t>(cdiv(n, kTileN) * cdiv(b, kTileM)));
  return v + 1;
}

int carve(Arena& a, int64_t m, int64_t n, int b, int64_t kcap, int power_iters, uint32_t flags,
          Work* w) {
  w->ldm = even_up(m);
  if (!(flags & QB_OVERWRITE_A)) {
    w->ldr = even_up(m);
    w->R = a.take<double>(static_cast<size_t>(w->ldr) * n);
  }
  w->omega = a.take<double>(static_cast<size_t>(n) * b);
  w->Y = a.take<double>(static_cast<size_t>(w->ldm) * b);
  w->Qi = a.take<double>(static_cast<size_t>(w->ldm) * b);
  if (power_iters > 0) w->Z = a.take<double>(static_cast<size_t>(n) * b);
  w->ldc = kcap > 0 ? kcap : 1;
  w->C = a.take<double>(static_cast<size_t>(w->ldc) * b);
  const bool exact = (flags & QB_SAMPLE_MASK) == QB_SAMPLE_INT8X8;
  w->part = a.take<double>(max_partials(m, n, b, kcap, exact));
  if (exact) w->omq = a.take<int8_t>(static_cast<size_t>(sample_i8_kp(n)) * b);
  const size_t nsq = max_sq(m, n, b);
  w->sq1 = a.take<double>(nsq);
  w->sq2 = a.take<double>(nsq);
  w->flags = a.take<int>(nsq);
  w->scal = a.take<double>(8);
  w->iscal = a.take<int>(4);
  int rc = orth_carve(a, std::max(m, n), b, &w->ow);
  if (a.base != nullptr && a.used > a.cap) return kEWorkspace;
  return rc;
}

// Sizes every kernel of the factorisation can launch: m x b and n x b
// panels (leading dimensions even_up(m) and n) below kMaxLd, and the
// downdate's column tiles within one grid dimension.
bool valid_sizes(int64_t m, int64_t n, int32_t b) {
  return m >= 1 && n >= 1 && b >= 1 && b <= kMaxPanel && even_up(m) < kMaxLd && n < kMaxLd &&
         n <= kMaxDowndateCols;
}

// Per-thread pinned host mailbox for the per-block scalars and an event that
// marks their arrival.  Pinned memory makes the device-to-host copy truly
// asynchronous, so work queued after it (the next block's sketch and
// sample) runs while the host waits only for the copy.  Allocated on first
// use and kept for the life of the thread (a few dozen bytes).
struct Mailbox {
  double* scal = nullptr;   // [0..1] resid^2 (hi, lo), [2..3] ||B_i||^2 (hi, lo)
  int* kept = nullptr;
  hipEvent_t ev = nullptr;
  bool ok = false;
};

Mailbox* mailbox() {
  thread_local Mailbox mb;
  if (!mb.ok) {
    void* p = nullptr;
    if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&mb.ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(p);
      return nullptr;
    }
    mb.scal = static_cast<double*>(p);
    mb.kept = reinterpret_cast<int*>(static_cast<char*>(p) + 4 * sizeof(double));
    mb.ok = true;
  }
  return &mb;
}

// Y = X W in the sampling precision.  QB_SAMPLE_INT8X8: the exact-range
// product of the quantised W with X on its fixed-point grid, the exponent
// taken from the device scalar *xnorm2 (||X||_F^2); omq holds the int8 W.
int sample(uint32_t prec, const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y,
           int64_t ldy, int64_t M, int64_t N, int64_t K, double* part, hipStream_t s,
           const double* xnorm2 = nullptr, int8_t* omq = nullptr) {
  if (prec == QB_SAMPLE_INT8X8) {
    if (xnorm2 == nullptr || omq == nullptr) return kEInval;
    if (quantize_sketch(W, ldw, K, static_cast<int>(N), omq, s)) return kEHip;
    return sample_i8(X, ldx, omq, Y, ldy, M, static_cast<int>(N), K, xnorm2, 0, part, s);
  }
  if (prec == QB_SAMPLE_F64)
    return gemm_nn(X, ldx, W, ldw, Y, ldy, M, N, K, 1.0, 0.0, choose_split(M, N, K, 2, true), part,
                   s);
  const int lp = prec == QB_SAMPLE_F32 ? 1 : 2;
  return gemm_nn_lowp(lp, X, ldx, W, ldw, Y, ldy, M, N, K, lowp_split(lp, true, M, N, K), part, s);
}

int project_t(uint32_t prec, const double* Qm, int64_t ldq, const double* X, int64_t ldx,
              double* C, int64_t ldc, int64_t P, int64_t N, int64_t K, bool tr, double* part,
              double* sq, int* sqc, hipStream_t s) {
  if (prec == QB_SAMPLE_F64)
    return gemm_tn(Qm, ldq, X, ldx, C, ldc, P, N, K, tr, choose_split(P, N, K), part, sq, sqc, s);
  const int lp = prec == QB_SAMPLE_F32 ? 1 : 2;
  return gemm_tn_lowp(lp, Qm, ldq, X, ldx, C, ldc, P, N, K, tr, lowp_split(lp, false, P, N, K),
                      part, s);
}

}  // namespace

int device_ready() {
  constexpr int kMaxDevices = 64;
  static std::atomic<signed char> known[kMaxDevices];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    (void)hipGetLastError();
    return kENoDevice;
  }
  signed char v = dev < kMaxDevices ? known[dev].load(std::memory_order_relaxed) : 0;
  if (v == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
      (void)hipGetLastError();
      return kENoDevice;
    }
    v = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    if (dev < kMaxDevices) known[dev].store(v, std::memory_order_relaxed);
  }
  return v > 0 ? kOk : kENoDevice;
}

}  // namespace qb

using namespace qb;

extern "C" {

const char* qb_status_string(int status) {
  switch (status) {
    case QB_OK: return "QB_OK";
    case QB_KMAX: return "QB_KMAX: k reached kmax before the tolerance";
    case QB_RANK_EXHAUSTED: return "QB_RANK_EXHAUSTED: residual at rounding level or full rank";
    case QB_NOT_CONVERGED: return "QB_NOT_CONVERGED: Jacobi sweeps reached their cap";
    case QB_EINVAL: return "QB_EINVAL: invalid argument";
    case QB_ENONFINITE: return "QB_ENONFINITE: input holds NaN or Inf";
    case QB_EWORKSPACE: return "QB_EWORKSPACE: workspace missing or too small";
    case QB_EHIP: return "QB_EHIP: HIP runtime error";
    case QB_ENODEVICE: return "QB_ENODEVICE: no usable device";
    case QB_ETOOBIG:
      return "QB_ETOOBIG: the problem needs more workspace than qb_factor_noalloc's fixed scratch";
    default: return "QB_UNKNOWN";
  }
}

size_t qb_workspace_bytes(int64_t m, int64_t n, int32_t b, int64_t kmax, uint32_t flags) {
  if (!valid_sizes(m, n, b) || kmax > std::min(m, n)) return 0;
  const int64_t r = std::min(m, n);
  const int64_t kcap = (kmax < 0) ? r : std::min(kmax, r);
  Arena a{nullptr, 0, 0};
  Work w;
  carve(a, m, n, std::min<int64_t>(b, r), kcap, /*power_iters=*/1, flags, &w);
  return a.used + 256;
}

}  // extern "C"

namespace {

// The factorisation behind qb_factor and qb_factor_noalloc.  With `pinned`
// the per-block scalars go through the thread's pinned mailbox (allocated on
// its first use) and an event; without it they are copied into a host stack
// buffer and the stream is synchronised, so nothing is allocated.
int factor_impl(const double* A, int64_t m, int64_t n, int64_t lda, double eps, int32_t b,
                int32_t power_iters, uint64_t seed, double* Q, int64_t ldq, double* B,
                int64_t ldb, int64_t kmax, int64_t* k_out, qb_info* info, void* workspace,
                size_t ws_bytes, void* stream, uint32_t flags, bool pinned) {
  Range rcall("qb_factor");
  if (k_out) *k_out = 0;
  if (!k_out || !A || !Q || !B) return QB_EINVAL;
  if (!valid_sizes(m, n, b) || power_iters < 0 || !(eps >= 0.0) || !std::isfinite(eps))
    return QB_EINVAL;
  const uint32_t prec = flags & QB_SAMPLE_MASK;
  // the B precision in the sampling encoding (QB_BGEMM_x >> 2 == QB_SAMPLE_x)
  const uint32_t bprec = (flags & QB_BGEMM_MASK) >> 2;
  if (bprec == QB_SAMPLE_MASK) return QB_EINVAL;
  const bool power_orth = (flags & QB_POWER_NO_ORTH) == 0;
  // The product whose columns span Q_i decides whether Q_i lies in the
  // range of the residual.  With power iterations, the last R Z runs in
  // float64 whatever the sampling precision: a rounded product leaves in
  // Q_i a component outside range(R) of the product's relative accuracy,
  // which no later block removes once k reaches min(m, n) < m.  The
  // products before it only steer the subspace and keep the low precision.
  const uint32_t range_prec = QB_SAMPLE_F64;
  // the exact-range sample serves the first product only; the products of
  // the power iterations run in float64 in that mode
  const uint32_t pow_prec = prec == QB_SAMPLE_INT8X8 ? QB_SAMPLE_F64 : prec;
  const bool single_block = (flags & QB_SINGLE_BLOCK) != 0;
  const int64_t r = std::min(m, n);
  if (kmax > r) return QB_EINVAL;
  const int64_t kcap = (kmax < 0) ? r : kmax;
  if (lda < m || ldq < m || ldb < std::max<int64_t>(kcap, 1)) return QB_EINVAL;
  if (lda >= kMaxLd || ldq >= kMaxLd || ldb >= kMaxLd) return QB_EINVAL;
  if (workspace == nullptr) return QB_EWORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EINVAL;
  if (const int dv = device_ready()) return dv;
  const int bw = static_cast<int>(std::min<int64_t>(b, r));

  Work wk;
  Arena arena{static_cast<char*>(workspace), ws_bytes, 0};
  if (carve(arena, m, n, bw, kcap, power_iters, flags, &wk) != kOk) return QB_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);

  // ||A||_F^2 and the non-finite check
  int cnt = 0;
  if (sumsq_partials(A, lda, m, n, wk.sq1, &cnt, wk.flags, st)) return QB_EHIP;
  if (sum_partials_ex(wk.sq1, cnt, wk.flags, wk.scal + 4, wk.iscal, st)) return QB_EHIP;
  double hsA[2];
  int hbad = 0;
  if (hipMemcpyAsync(hsA, wk.scal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&hbad, wk.iscal, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QB_EHIP;
  if (hbad) return QB_ENONFINITE;
  if (!std::isfinite(hsA[0])) return QB_EINVAL;  // ||A||_F^2 overflows a double
  const DD sA{hsA[0], hsA[1]};
  const double sAv = dd_val(sA);
  const double eps2 = eps * eps;
  // hybrid band half-width: |E_i - D_i| grows to about 2 u ||A||^2 with the
  // unit roundoff u of the B product
  const double delta = (bprec == QB_SAMPLE_F64   ? kDeltaRel
                        : bprec == QB_SAMPLE_F32 ? kDeltaRelF32
                                                 : kDeltaRelBf16x3) * sAv;
  const double floor2 = (kFloorRel * std::sqrt(sAv)) * (kFloorRel * std::sqrt(sAv));

  int64_t k = 0;
  int blocks = 0;
  int reason = QB_STOP_ZERO;
  double lastE = sAv, lastD = sAv;
  auto finish = [&](int why) -> int {
    *k_out = k;
    if (info) {
      info->k = k;
      info->blocks = blocks;
      info->stop_reason = why;
      info->normA2 = sAv;
      info->indicator = lastE;
      info->resid2 = lastD;
    }
    if (why == QB_STOP_ZERO || why == QB_STOP_TOL_TRACKED || why == QB_STOP_TOL_DIRECT) return QB_OK;
    if (why == QB_STOP_KMAX) return QB_KMAX;
    return QB_RANK_EXHAUSTED;
  };
  if (info) info->trace_len = 0;
  if (sAv <= eps2) return finish(QB_STOP_ZERO);

  double* R;
  int64_t ldr;
  if (flags & QB_OVERWRITE_A) {
    R = const_cast<double*>(A);
    ldr = lda;
  } else {
    R = wk.R;
    ldr = wk.ldr;
    if (copy_matrix(A, lda, R, ldr, m, n, st)) return QB_EHIP;
  }

  Mailbox* mb = nullptr;
  double hbox[4] = {0.0, 0.0, 0.0, 0.0};
  int hkept = 0;
  if (pinned) {
    mb = mailbox();
    if (mb == nullptr) return QB_EHIP;
  }
  double* box_scal = mb ? mb->scal : hbox;
  int* box_kept = mb ? mb->kept : &hkept;
  DD sigB{0.0, 0.0};
  const int64_t ldm = wk.ldm;
  // sketch and sample of a block already queued behind the previous block's
  // scalars (started before the stop decision was known), as (k, w)
  int64_t spec_k = -1;
  int spec_w = 0;
  for (;;) {
    const int w = static_cast<int>(std::min<int64_t>(bw, kcap - k));
    if (w <= 0) { reason = (kcap < r) ? QB_STOP_KMAX : QB_STOP_RANK_CAP; break; }
    Range rblock("qb_block");
    // (2)-(3) sample the residual and orthonormalise
    if (spec_k != k || spec_w != w) {
      if (launch_sketch(seed, n, k, w, wk.omega, n, st)) return QB_EHIP;
      // ||R||_F^2 of the residual being sampled: ||A||^2, then D of the last block
      if (sample(prec, R, ldr, wk.omega, n, wk.Y, ldm, m, w, n, wk.part, st,
                 k == 0 ? wk.scal + 4 : wk.scal + 0, wk.omq))
        return QB_EHIP;
    }
    spec_k = -1;
    std::optional<Range> rsub;
    rsub.emplace("qb_block_range_finder");
    if (power_orth) {
      if (orth_cholqr2(wk.Y, ldm, wk.Qi, ldm, m, w, wk.ow, st)) return QB_EHIP;
      // (4)-(7) power iterations on the residual
      for (int p = 0; p < power_iters; ++p) {
        if (project_t(pow_prec, wk.Qi, ldm, R, ldr, wk.Z, n, w, n, m, true, wk.part, nullptr,
                      nullptr, st))
          return QB_EHIP;
        if (orth_cholqr2(wk.Z, n, wk.Z, n, n, w, wk.ow, st)) return QB_EHIP;
        if (sample(p + 1 == power_iters ? range_prec : pow_prec, R, ldr, wk.Z, n, wk.Y, ldm, m, w,
                   n, wk.part, st))
          return QB_EHIP;
        if (orth_cholqr2(wk.Y, ldm, wk.Qi, ldm, m, w, wk.ow, st)) return QB_EHIP;
      }
    } else {
      // Section 5.4: Y = (R R^T)^P R Omega_i without intermediate orth
      for (int p = 0; p < power_iters; ++p) {
        if (project_t(pow_prec, wk.Y, ldm, R, ldr, wk.Z, n, w, n, m, true, wk.part, nullptr, nullptr,
                      st))
          return QB_EHIP;
        if (sample(p + 1 == power_iters ? range_prec : pow_prec, R, ldr, wk.Z, n, wk.Y, ldm, m, w,
                   n, wk.part, st))
          return QB_EHIP;
      }
      if (orth_cholqr2(wk.Y, ldm, wk.Qi, ldm, m, w, wk.ow, st)) return QB_EHIP;
    }
    rsub.reset();
    rsub.emplace("qb_block_reproject_B_downdate");
    double* Qout = Q + k * ldq;
    // (3') re-projection against the basis so far, then orth
    if (k > 0) {
      const int sp = choose_split(w, k, m);
      if (gemm_tn(wk.Qi, ldm, Q, ldq, wk.C, wk.ldc, w, k, m, true, sp, wk.part, nullptr, nullptr, st))
        return QB_EHIP;
      const int sq = choose_split(m, w, k, 2, true);
      if (gemm_nn(Q, ldq, wk.C, wk.ldc, wk.Qi, ldm, m, w, k, -1.0, 1.0, sq, wk.part, st))
        return QB_EHIP;
      if (orth_cholqr2(wk.Qi, ldm, Qout, ldq, m, w, wk.ow, st)) return QB_EHIP;
    } else {
      if (copy_matrix(wk.Qi, ldm, Qout, ldq, m, w, st)) return QB_EHIP;
    }
    // (4) B_i = Q_i^T A with ||B_i||^2;  (5) downdate with ||A^(i)||^2
    int nb = 0, nd = 0;
    if (bprec == QB_SAMPLE_F64) {
      const int sp = choose_split(w, n, m);
      if (gemm_tn(Qout, ldq, R, ldr, B + k, ldb, w, n, m, false, sp, wk.part, wk.sq1, &nb, st))
        return QB_EHIP;
    } else {
      if (project_t(bprec, Qout, ldq, R, ldr, B + k, ldb, w, n, m, false, wk.part, nullptr,
                    nullptr, st))
        return QB_EHIP;
      if (sumsq_partials(B + k, ldb, w, n, wk.sq1, &nb, wk.flags, st)) return QB_EHIP;
    }
    if (sum_partials(wk.sq1, nb, wk.scal + 2, st)) return QB_EHIP;
    if (downdate(R, ldr, Qout, ldq, B + k, ldb, m, n, w, wk.sq2, &nd, st)) return QB_EHIP;
    if (sum_partials(wk.sq2, nd, wk.scal + 0, st)) return QB_EHIP;
    if (hipMemcpyAsync(box_scal, wk.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(box_kept, wk.ow.kept, sizeof(int), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        (mb && hipEventRecord(mb->ev, st) != hipSuccess))
      return QB_EHIP;
    // Queue the next block's sketch and sample (they read only R, already
    // downdated, and write only Omega and Y) assuming no column is dropped;
    // the host decides meanwhile.  After a stop they are left unused.
    {
      const int64_t kn = k + w;
      const int wn = static_cast<int>(std::min<int64_t>(bw, kcap - kn));
      if (wn > 0 && !single_block && !(flags & QB_NO_SPECULATE)) {
        if (launch_sketch(seed, n, kn, wn, wk.omega, n, st)) return QB_EHIP;
        if (sample(prec, R, ldr, wk.omega, n, wk.Y, ldm, m, wn, n, wk.part, st, wk.scal + 0,
                   wk.omq))
          return QB_EHIP;
        spec_k = kn;
        spec_w = wn;
      }
    }
    if ((mb ? hipEventSynchronize(mb->ev) : hipStreamSynchronize(st)) != hipSuccess)
      return QB_EHIP;
    double hs[4];
    std::memcpy(hs, box_scal, sizeof(hs));
    const int wkept = *box_kept;
    if (wkept <= 0) { reason = QB_STOP_EXHAUSTED; break; }
    k += wkept;
    ++blocks;
    sigB = dd_add(sigB, DD{hs[2], hs[3]});
    const DD Edd = dd_add(sA, DD{-sigB.hi, -sigB.lo});
    lastE = dd_val(Edd);
    lastD = hs[0] + hs[1];
    if (info && info->trace_cap > info->trace_len) {
      const int t = info->trace_len++;
      if (info->trace_w) info->trace_w[t] = wkept;
      if (info->trace_E) info->trace_E[t] = lastE;
      if (info->trace_D) info->trace_D[t] = lastD;
    }
    // (6) stopping rule
    if (lastE <= eps2 - delta) { reason = QB_STOP_TOL_TRACKED; break; }
    if (!(lastE > eps2 + delta) && lastD <= eps2) { reason = QB_STOP_TOL_DIRECT; break; }
    if (lastD <= floor2) { reason = QB_STOP_EXHAUSTED; break; }
    if (single_block) { reason = QB_STOP_KMAX; break; }
    if (k >= kcap) { reason = (kcap < r) ? QB_STOP_KMAX : QB_STOP_RANK_CAP; break; }
  }
  return finish(reason);
}

// Fixed device scratch of qb_factor_noalloc: one copy per device, held from
// the library's load until the process ends.  Host code never uses the
// symbol's name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
__device__ __align__(256) char scratch[QB_NOALLOC_SCRATCH_BYTES];

void* scratch_address() {
  constexpr int kMaxDevices = 64;
  static std::atomic<void*> addr[kMaxDevices];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  void* p = addr[dev].load(std::memory_order_acquire);
  if (p == nullptr) {
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    addr[dev].store(p, std::memory_order_release);  // same value from any racing thread
  }
  return p;
}

}  // namespace

extern "C" {

int qb_factor(const double* A, int64_t m, int64_t n, int64_t lda, double eps, int32_t b,
              int32_t power_iters, uint64_t seed, double* Q, int64_t ldq, double* B, int64_t ldb,
              int64_t kmax, int64_t* k_out, qb_info* info, void* workspace, size_t ws_bytes,
              void* stream, uint32_t flags) {
  return factor_impl(A, m, n, lda, eps, b, power_iters, seed, Q, ldq, B, ldb, kmax, k_out, info,
                     workspace, ws_bytes, stream, flags, /*pinned=*/true);
}

int qb_factor_noalloc(const double* A, int64_t m, int64_t n, int64_t lda, double eps, int32_t b,
                      int32_t power_iters, uint64_t seed, double* Q, int64_t ldq, double* B,
                      int64_t ldb, int64_t kmax, int64_t* k_out, qb_info* info, void* stream,
                      uint32_t flags) {
  if (k_out) *k_out = 0;
  const size_t need = qb_workspace_bytes(m, n, b, kmax, flags);
  if (need == 0) return QB_EINVAL;
  if (need > QB_NOALLOC_SCRATCH_BYTES) return QB_ETOOBIG;
  if (const int dv = device_ready()) return dv;
  void* ws = scratch_address();
  if (ws == nullptr) return QB_EHIP;
  return factor_impl(A, m, n, lda, eps, b, power_iters, seed, Q, ldq, B, ldb, kmax, k_out, info,
                     ws, QB_NOALLOC_SCRATCH_BYTES, stream, flags, /*pinned=*/false);
}

int qb_sketch(uint64_t seed, int64_t n, int64_t col0, int32_t w, double* out, int64_t ld,
              void* stream) {
  if (!out || n < 1 || w < 1 || col0 < 0 || ld < n || col0 + w > (int64_t(1) << 32))
    return QB_EINVAL;
  if (const int dv = device_ready()) return dv;
  return launch_sketch(seed, n, col0, w, out, ld, static_cast<hipStream_t>(stream)) ? QB_EHIP
                                                                                    : QB_OK;
}

size_t qb_orth_workspace_bytes(int64_t m, int32_t w) {
  if (m < 1 || w < 1 || w > kMaxPanel) return 0;
  return orth_work_bytes(m, w);
}

int qb_orth(const double* X, int64_t m, int32_t w, int64_t ldx, double* Q, int64_t ldq,
            int32_t* kept, void* workspace, size_t ws_bytes, void* stream) {
  if (kept) *kept = 0;
  if (!X || !Q || m < 1 || w < 1 || w > kMaxPanel || ldx < m || ldq < m) return QB_EINVAL;
  if (even_up(m) >= kMaxLd || ldx >= kMaxLd || ldq >= kMaxLd) return QB_EINVAL;
  if (Q == X && ldq != ldx) return QB_EINVAL;
  if (!workspace) return QB_EWORKSPACE;
  if (const int dv = device_ready()) return dv;
  Arena a{static_cast<char*>(workspace), ws_bytes, 0};
  OrthWork ow;
  if (orth_carve(a, m, w, &ow) != kOk) return QB_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (orth_cholqr2(X, ldx, Q, ldq, m, w, ow, st)) return QB_EHIP;
  int hk = 0;
  if (hipMemcpyAsync(&hk, ow.kept, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QB_EHIP;
  if (kept) *kept = hk;
  return QB_OK;
}

}  // extern "C"

namespace {
// Workspace of qb_sample / qb_project: split-K partials (float64 and the
// exact-range form), the int8 sketch, and the ||X||_F^2 pass of the exact
// form (per-workgroup sums, flags, scalars).
struct GemmScratch {
  double* part = nullptr;
  int8_t* omq = nullptr;
  double* sq = nullptr;
  int* fl = nullptr;
  double* scal = nullptr;
  int* iscal = nullptr;
};
size_t gemm_scratch(void* workspace, size_t ws_bytes, int64_t m, int64_t K, int32_t w,
                    GemmScratch* g) {
  Arena a{static_cast<char*>(workspace), ws_bytes, 0};
  // the sample Y (m x w, depth K) in every precision, and the projection
  // C (w x m, depth K) with the splits project_t takes
  size_t np = std::max(partial_doubles(m, w, choose_split(m, w, K, 2, true)),
                       std::max(partial_doubles(m, w, choose_split(m, w, K, 2, false)),
                                sample_i8_partials(m, w, K)));
  np = std::max(np, partial_doubles(w, m, choose_split(w, m, K)));
  for (int lp : {1, 2}) {
    np = std::max(np, lowp_scratch_doubles(lp, true, m, w, K));
    np = std::max(np, lowp_scratch_doubles(lp, false, w, m, K));
  }
  g->part = a.take<double>(np + 1);
  g->omq = a.take<int8_t>(static_cast<size_t>(sample_i8_kp(K)) * w);
  const size_t nsq = sumsq_partials_count(m, K) + 1;
  g->sq = a.take<double>(nsq);
  g->fl = a.take<int>(nsq);
  g->scal = a.take<double>(8);
  g->iscal = a.take<int>(4);
  return a.used;
}
}  // namespace

extern "C" {

size_t qb_gemm_workspace_bytes(int64_t m, int64_t K, int32_t w) {
  if (m < 1 || K < 0 || w < 1 || w > kMaxPanel) return 0;
  GemmScratch g;
  return gemm_scratch(nullptr, 0, m, K, w, &g);
}

int qb_sample(const double* X, int64_t m, int64_t K, int64_t ldx, const double* W, int32_t w,
              int64_t ldw, double* Y, int64_t ldy, uint32_t precision, void* workspace,
              size_t ws_bytes, void* stream) {
  if (!X || !W || !Y || m < 1 || K < 1 || w < 1 || w > kMaxPanel || ldx < m || ldw < K || ldy < m)
    return QB_EINVAL;
  if (ldx >= kMaxLd || ldw >= kMaxLd || ldy >= kMaxLd) return QB_EINVAL;
  if (precision != QB_SAMPLE_F64 && precision != QB_SAMPLE_F32 &&
      precision != QB_SAMPLE_BF16X3 && precision != QB_SAMPLE_INT8X8)
    return QB_EINVAL;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EWORKSPACE;
  GemmScratch g;
  if (gemm_scratch(workspace, ws_bytes, m, K, w, &g) > ws_bytes) return QB_EWORKSPACE;
  if (const int dv = device_ready()) return dv;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (precision == QB_SAMPLE_INT8X8) {
    int cnt = 0;  // ||X||_F^2 fixes the fixed-point grid
    if (sumsq_partials(X, ldx, m, K, g.sq, &cnt, g.fl, st)) return QB_EHIP;
    if (sum_partials_ex(g.sq, cnt, g.fl, g.scal, g.iscal, st)) return QB_EHIP;
  }
  return sample(precision, X, ldx, W, ldw, Y, ldy, m, w, K, g.part, st, g.scal, g.omq) ? QB_EHIP
                                                                                     : QB_OK;
}

int qb_project(const double* Qm, int64_t K, int32_t w, int64_t ldq, const double* X, int64_t N,
               int64_t ldx, double* C, int64_t ldc, uint32_t precision, void* workspace,
               size_t ws_bytes, void* stream) {
  if (!Qm || !X || !C || K < 1 || N < 1 || w < 1 || w > kMaxPanel || ldq < K || ldx < K || ldc < w)
    return QB_EINVAL;
  if (ldq >= kMaxLd || ldx >= kMaxLd || ldc >= kMaxLd) return QB_EINVAL;
  if (precision != QB_SAMPLE_F64 && precision != QB_SAMPLE_F32 && precision != QB_SAMPLE_BF16X3)
    return QB_EINVAL;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return QB_EWORKSPACE;
  GemmScratch g;
  if (gemm_scratch(workspace, ws_bytes, N, K, w, &g) > ws_bytes) return QB_EWORKSPACE;
  if (const int dv = device_ready()) return dv;
  return project_t(precision, Qm, ldq, X, ldx, C, ldc, w, N, K, false, g.part, nullptr, nullptr,
                   static_cast<hipStream_t>(stream)) ? QB_EHIP : QB_OK;
}

size_t qb_downdate_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1) return 0;
  const size_t v = std::max(downdate_partials(m, n), sumsq_partials_count(m, n)) + 1;
  return v * (sizeof(double) + sizeof(int)) + 8 * sizeof(double) + 4 * 256;
}

static int small_scratch(void* workspace, size_t ws_bytes, int64_t m, int64_t n, double** sq,
                         int** fl, double** scal, int** iscal) {
  const size_t v = std::max(downdate_partials(m, n), sumsq_partials_count(m, n)) + 1;
  Arena a{static_cast<char*>(workspace), ws_bytes, 0};
  *sq = a.take<double>(v);
  *fl = a.take<int>(v);
  *scal = a.take<double>(8);
  *iscal = a.take<int>(4);
  return a.used > a.cap ? QB_EWORKSPACE : QB_OK;
}

int qb_downdate(double* R, int64_t m, int64_t n, int64_t ldr, const double* Qm, int32_t w,
                int64_t ldq, const double* B, int64_t ldb, double* resid2, void* workspace,
                size_t ws_bytes, void* stream) {
  if (!R || !Qm || !B || m < 1 || n < 1 || w < 1 || ldr < m || ldq < m || ldb < w)
    return QB_EINVAL;
  if (ldq >= kMaxLd || ldb >= kMaxLd || n > kMaxDowndateCols) return QB_EINVAL;
  if (!workspace) return QB_EWORKSPACE;
  double *sq, *scal;
  int *fl, *iscal;
  if (small_scratch(workspace, ws_bytes, m, n, &sq, &fl, &scal, &iscal)) return QB_EWORKSPACE;
  if (const int dv = device_ready()) return dv;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int cnt = 0;
  if (downdate(R, ldr, Qm, ldq, B, ldb, m, n, w, sq, &cnt, st)) return QB_EHIP;
  if (resid2) {
    if (sum_partials(sq, cnt, scal, st)) return QB_EHIP;
    double h[2];
    if (hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QB_EHIP;
    *resid2 = h[0] + h[1];
  }
  return QB_OK;
}

int qb_frob2(const double* X, int64_t m, int64_t n, int64_t ldx, double* out, int32_t* nonfinite,
             void* workspace, size_t ws_bytes, void* stream) {
  if (!X || !out || m < 1 || n < 1 || ldx < m) return QB_EINVAL;
  if (!workspace) return QB_EWORKSPACE;
  double *sq, *scal;
  int *fl, *iscal;
  if (small_scratch(workspace, ws_bytes, m, n, &sq, &fl, &scal, &iscal)) return QB_EWORKSPACE;
  if (const int dv = device_ready()) return dv;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int cnt = 0;
  if (sumsq_partials(X, ldx, m, n, sq, &cnt, fl, st)) return QB_EHIP;
  if (sum_partials_ex(sq, cnt, fl, scal, iscal, st)) return QB_EHIP;
  double h[2];
  int bad = 0;
  if (hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&bad, iscal, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QB_EHIP;
  *out = h[0] + h[1];
  if (nonfinite) *nonfinite = bad;
  return QB_OK;
}

}  // extern "C"
