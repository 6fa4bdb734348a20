// Exact-range sampling product on the int8 MFMA (gfx950).
//
// The sample Y = A Omega_i of Figure 4 step (3) spans Q_i.  A rounded
// low-precision product leaves a component outside range(A) in Q_i, and
// once the rank reaches min(m, n) < m no later block removes it.  This
// product is exact instead, on integers:
//
//   Omega~ = clip(rint(16 Omega), -127, 127) / 16      (int8, k-contiguous)
//   E      = ceil(e / 2) + 1 with ||A||_F^2 = f 2^e, f in [1/2, 1), so every
//            entry of A lies below 2^(E-1)
//   v      = rint(a 2^(55-E)) for each entry a: an integer, |v| < 2^54,
//            held as eight base-128 digits (seven 7-bit fields and a signed
//            top field), each an int8
//   Y      = 2^(E-59) sum_s 128^s (D_s Omega~q)
//
// where D_s holds digit s of every entry and Omega~q = 16 Omega~.  Each
// digit product D_s Omega~q is summed exactly in int32 by
// v_mfma_i32_16x16x64_i8 (|digit| <= 127, |Omega~q| <= 127, depth chunks of
// at most 2^17), and the eight sums are combined in float64.  So Y is the
// float64 rounding of A~ Omega~ with A~ within 2^(E-56) of A per entry: as
// close to range(A) as a float64 product.
//
// Work split: a workgroup owns 32 rows and all w (<= 256) columns of Y for
// one depth chunk, so every entry of A is read from HBM and split into
// digits exactly once per chunk.  Depth steps of 64 pass through two LDS
// stages: the digits of a 32 x 64 tile of A (8 slices of 32 x 64 bytes) and
// the 64 x w sketch tile; the next step's A entries and sketch bytes are in
// registers meanwhile.  Waves are 2 (rows) x w/64 (columns); each owns
// 16 x 64 of Y as four 16 x 16 MFMA blocks per digit (128 int32
// accumulators per lane).  Chunks of a split depth write float64 partials
// that a second kernel adds in chunk order.
#include <cfloat>

#include "qb_internal.hpp"

namespace qb {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kDigits = 8;
constexpr int kStep = 64;        // depth per MFMA
constexpr int kRows = 32;        // rows of Y per workgroup
constexpr int kLdsRow = 80;      // bytes per LDS row (64 + 16: 16-byte aligned, staggered banks)
constexpr int kFracBits = 55;
constexpr int64_t kMaxChunk = int64_t(1) << 17;  // 127 * 127 * 2^17 < 2^31

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// row of the 16 x 16 result held in element r of lane l
#define I8_ROW(l, r) (4 * ((l) >> 4) + (r))

__device__ __forceinline__ int split_exponent_dev(double D) {
  if (!(D > 0.0) || !(D <= DBL_MAX)) return 0;
  int e;
  (void)frexp(D, &e);
  return -((-e) >> 1) + 1;  // ceil(e / 2) + 1
}

// Omega (n x w, ld) -> int8 [column][k] with leading dimension kp (a
// multiple of 64), rows n .. kp-1 zero.  Four bytes per thread.
__global__ __launch_bounds__(256) void quantize_sketch_kernel(const double* __restrict__ om,
                                                              int64_t ldo, int64_t n, int w,
                                                              int8_t* __restrict__ q,
                                                              int64_t kp) {
  const int64_t quad = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t per_col = kp / 4;
  if (quad >= per_col * w) return;
  const int64_t j = quad / per_col, k0 = 4 * (quad % per_col);
  uint32_t word = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int v = 0;
    if (k0 + c < n) {
      double x = rint(om[k0 + c + j * ldo] * 16.0);
      x = x > 127.0 ? 127.0 : (x < -127.0 ? -127.0 : x);
      v = static_cast<int>(x);
    }
    word |= (static_cast<uint32_t>(v) & 255u) << (8 * c);
  }
  *reinterpret_cast<uint32_t*>(q + k0 + j * kp) = word;
}

// four 7-bit fields of v (bits 0..27) into the four bytes
__device__ __forceinline__ uint32_t spread_lo(uint32_t v) {
  uint32_t r = v & 0x7fu;
  r = ((v << 1) & 0x7f00u) | r;
  r = ((v << 2) & 0x7f0000u) | r;
  return ((v << 3) & 0x7f000000u) | r;
}
// three 7-bit fields of v and its signed top field (bits 21..28, the sign
// extension of v >> 21) into the four bytes
__device__ __forceinline__ uint32_t spread_hi(uint32_t v) {
  uint32_t r = v & 0x7fu;
  r = ((v << 1) & 0x7f00u) | r;
  r = ((v << 2) & 0x7f0000u) | r;
  return ((v << 3) & 0xff000000u) | r;
}
// 4 x 4 byte transpose: d[s] byte c = w[c] byte s (v_perm_b32 picks bytes
// 0..3 of its second operand with selectors 0..3, of its first with 4..7)
__device__ __forceinline__ void transpose4(const uint32_t (&w)[4], uint32_t* d) {
  const uint32_t x0 = __builtin_amdgcn_perm(w[1], w[0], 0x06020400u);
  const uint32_t x1 = __builtin_amdgcn_perm(w[1], w[0], 0x07030501u);
  const uint32_t y0 = __builtin_amdgcn_perm(w[3], w[2], 0x06020400u);
  const uint32_t y1 = __builtin_amdgcn_perm(w[3], w[2], 0x07030501u);
  d[0] = __builtin_amdgcn_perm(y0, x0, 0x05040100u);
  d[2] = __builtin_amdgcn_perm(y0, x0, 0x07060302u);
  d[1] = __builtin_amdgcn_perm(y1, x1, 0x05040100u);
  d[3] = __builtin_amdgcn_perm(y1, x1, 0x07060302u);
}

// digits of four entries of one row at consecutive depths, packed one
// dword per digit (byte c = entry c): v = rint(x 2^(55-E)) = h 2^28 + l
// with 0 <= l < 2^28; digits 0..3 are the 7-bit fields of l, digits 4..6
// those of h, digit 7 the signed h >> 21
__device__ __forceinline__ void digits4(const double (&x)[4], double scale, uint32_t (&out)[kDigits]) {
  uint32_t wl[4], wh[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double t = rint(x[c] * scale);          // |t| < 2^54, exact scaling
    const double h = floor(t * 0x1p-28);          // exact
    const double l = fma(-h, 0x1p28, t);          // exact, in [0, 2^28)
    wh[c] = spread_hi(static_cast<uint32_t>(static_cast<int>(h)));
    wl[c] = spread_lo(static_cast<uint32_t>(static_cast<int>(l)));
  }
  transpose4(wl, out);
  transpose4(wh, out + 4);
}

// Y (M x N, N <= BN) for rows [32 bx, +32) and depth chunk z.  dnorm2: the
// device ||A||_F^2 that fixes E, or null to use e_host.
template <int BN>
__global__ __launch_bounds__(2 * BN, 1) void sample_i8_kernel(
    const double* __restrict__ A, int64_t lda, const int8_t* __restrict__ q, int64_t kp,
    double* __restrict__ Y, int64_t ldy, int64_t M, int N, int64_t K, int64_t kchunk,
    const double* __restrict__ dnorm2, int e_host, double* __restrict__ part, int64_t ldp,
    int tiles_chunks) {
  constexpr int NT = 2 * BN;
  constexpr int UPT = (kRows * kStep / 4) / NT;   // 4-entry units per thread per step
  constexpr int BPT = (BN * kStep / 16) / NT;     // 16-byte sketch pieces per thread per step
  constexpr int A_STAGE = kDigits * kRows * kLdsRow;
  constexpr int B_STAGE = BN * kLdsRow;
  __shared__ __attribute__((aligned(16))) int8_t As[2 * A_STAGE];
  __shared__ __attribute__((aligned(16))) int8_t Bs[2 * B_STAGE];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave & 1) * 16, wn = (wave >> 1) * 64;
  // XCD-aware order: workgroup L runs on XCD L mod 8; XCD x takes a
  // contiguous run of (chunk, row tile) pairs, so the workgroups resident on
  // one XCD read neighbouring 256-byte row segments of the same columns of
  // A (whole DRAM pages between them) instead of segments 8 tiles apart.
  int64_t tile, chunk;
  {
    constexpr int kXcd = 8;
    const int64_t tiles_m = gridDim.x / tiles_chunks;
    const int64_t L = blockIdx.x, total = gridDim.x;
    const int64_t q = total / kXcd, r = total % kXcd, x = L % kXcd, j = L / kXcd;
    const int64_t logical = x * q + (x < r ? x : r) + j;
    chunk = logical / tiles_m;
    tile = logical - chunk * tiles_m;
  }
  const int64_t m0 = tile * kRows;
  const int64_t kbeg = chunk * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const int E = dnorm2 ? split_exponent_dev(dnorm2[0]) : e_host;
  const double scale = ldexp(1.0, kFracBits - E);

  // per-thread load assignment: unit u = t + NT * p -> row u % 32, depth quad u / 32
  int urow[UPT], ukq[UPT];
#pragma unroll
  for (int p = 0; p < UPT; ++p) {
    const int u = t + NT * p;
    urow[p] = u % kRows;
    ukq[p] = u / kRows;
  }
  double ra[UPT][4];
  i32x4 rb[BPT];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < UPT; ++p) {
      const int64_t row = m0 + urow[p];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t k = k0 + 4 * ukq[p] + c;
        ra[p][c] = (row < M && k < kend) ? A[row + k * lda] : 0.0;
      }
    }
#pragma unroll
    for (int p = 0; p < BPT; ++p) {
      const int piece = t + NT * p;
      const int col = piece >> 2, part16 = piece & 3;
      rb[p] = (col < N) ? *reinterpret_cast<const i32x4*>(q + k0 + 16 * part16 + col * kp)
                        : (i32x4){0, 0, 0, 0};
    }
  };
  auto store = [&](int stage) {
    int8_t* as = As + stage * A_STAGE;
    int8_t* bs = Bs + stage * B_STAGE;
#pragma unroll
    for (int p = 0; p < UPT; ++p) {
      uint32_t dg[kDigits];
      digits4(ra[p], scale, dg);
#pragma unroll
      for (int s = 0; s < kDigits; ++s)
        *reinterpret_cast<uint32_t*>(as + s * kRows * kLdsRow + urow[p] * kLdsRow + 4 * ukq[p]) =
            dg[s];
    }
#pragma unroll
    for (int p = 0; p < BPT; ++p) {
      const int piece = t + NT * p;
      const int col = piece >> 2, part16 = piece & 3;
      *reinterpret_cast<i32x4*>(bs + col * kLdsRow + 16 * part16) = rb[p];
    }
  };

  i32x4 acc[kDigits][4];
#pragma unroll
  for (int s = 0; s < kDigits; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[s][j] = (i32x4){0, 0, 0, 0};

  const int nsteps = static_cast<int>(cdiv(kend - kbeg, kStep));
  const bool active_cols = wn < N;  // waves right of the panel only stage data
  if (nsteps > 0) {
    load(kbeg);
    store(0);
    if (nsteps > 1) load(kbeg + kStep);
    lds_barrier();
    int stage = 0;
    for (int st = 0; st < nsteps; ++st) {
      if (st + 1 < nsteps) {
        store(stage ^ 1);
        if (st + 2 < nsteps) load(kbeg + static_cast<int64_t>(st + 2) * kStep);
      }
      if (active_cols) {
        const int8_t* as = As + stage * A_STAGE;
        const int8_t* bs = Bs + stage * B_STAGE;
        const int fr = lane & 15, fk = 16 * (lane >> 4);
        i32x4 b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[j] = *reinterpret_cast<const i32x4*>(bs + (wn + 16 * j + fr) * kLdsRow + fk);
#pragma unroll
        for (int s = 0; s < kDigits; ++s) {
          const i32x4 a =
              *reinterpret_cast<const i32x4*>(as + s * kRows * kLdsRow + (wm + fr) * kLdsRow + fk);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[s][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b[j], acc[s][j], 0, 0, 0);
        }
      }
      lds_barrier();
      stage ^= 1;
    }
  }
  if (!active_cols) return;

  // combine the digit sums: y = sum_s 128^s acc_s, then scale by 2^(E-59)
  const double oscale = ldexp(1.0, E - kFracBits - 4);
  double* out = part ? part + chunk * ldp * N : Y;
  const int64_t ldo = part ? ldp : ldy;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = wn + 16 * j + (lane & 15);
    if (col >= N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + wm + I8_ROW(lane, r);
      double y = static_cast<double>(acc[kDigits - 1][j][r]);
#pragma unroll
      for (int s = kDigits - 2; s >= 0; --s) y = fma(y, 128.0, static_cast<double>(acc[s][j][r]));
      if (row < M) out[row + col * ldo] = y * oscale;
    }
  }
}

// ordered sum of the depth chunks' partials
__global__ __launch_bounds__(256) void i8_reduce_kernel(const double* __restrict__ part, int nz,
                                                        int64_t ldp, double* __restrict__ Y,
                                                        int64_t ldy, int64_t M, int64_t N) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx % M, j = idx / M;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += part[i + j * ldp + static_cast<int64_t>(z) * ldp * N];
  Y[i + j * ldy] = s;
}

}  // namespace

int64_t sample_i8_kp(int64_t K) { return cdiv(K, kStep) * kStep; }

int sample_i8_split(int64_t M, int64_t K) {
  // about four workgroups per CU over the row tiles and chunks, chunks of
  // at least 1024 and at most 2^17 deep
  const int64_t tiles = cdiv(M, kRows);
  int64_t nz = cdiv(int64_t(4) * kNumCU, tiles);
  const int64_t by_depth = K / 1024;
  if (nz > by_depth) nz = by_depth;
  if (nz < cdiv(K, kMaxChunk)) nz = cdiv(K, kMaxChunk);
  if (nz < 1) nz = 1;
  if (nz > kMaxSplit) nz = kMaxSplit;
  return static_cast<int>(nz);
}

size_t sample_i8_partials(int64_t M, int64_t N, int64_t K) {
  const int nz = sample_i8_split(M, K);
  return nz > 1 ? static_cast<size_t>((M + 1) & ~int64_t(1)) * N * nz : 0;
}

int quantize_sketch(const double* om, int64_t ldo, int64_t n, int w, int8_t* q, hipStream_t s) {
  const int64_t kp = sample_i8_kp(n);
  const int64_t quads = (kp / 4) * w;
  ProfScope ps(kKSketch, 0.0, 9.0 * n * w, s);
  hipLaunchKernelGGL(quantize_sketch_kernel, dim3(static_cast<unsigned>(cdiv(quads, 256))),
                     dim3(256), 0, s, om, ldo, n, w, q, kp);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int sample_i8(const double* A, int64_t lda, const int8_t* q, double* Y, int64_t ldy, int64_t M,
              int N, int64_t K, const double* dnorm2, int e_host, double* part, hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  if (N > 256 || K <= 0 || M >= (int64_t(1) << 31) / kRows) return kEInval;
  const int64_t kp = sample_i8_kp(K);
  const int nz = sample_i8_split(M, K);
  const int64_t kc = sample_i8_kp(cdiv(K, nz));
  const int nzr = static_cast<int>(cdiv(K, kc));
  if (kc > kMaxChunk) return kEInval;
  if (cdiv(M, kRows) * nzr >= (int64_t(1) << 31)) return kEInval;  // one-dimensional grid
  if (nzr > 1 && part == nullptr) return kEInval;
  const int64_t ldp = (M + 1) & ~int64_t(1);
  double* pp = nzr > 1 ? part : nullptr;
  // one-dimensional grid: (row tile, depth chunk) pairs, chunk-major
  const dim3 grid(static_cast<unsigned>(cdiv(M, kRows) * nzr));
  {
    ProfScope ps(kKSampleI8, 2.0 * M * N * K, 8.0 * M * K + 1.0 * K * N + 8.0 * M * N, s);
    if (N <= 64)
      hipLaunchKernelGGL(sample_i8_kernel<64>, grid, dim3(128), 0, s, A, lda, q, kp, Y, ldy, M, N,
                         K, kc, dnorm2, e_host, pp, ldp, nzr);
    else if (N <= 128)
      hipLaunchKernelGGL(sample_i8_kernel<128>, grid, dim3(256), 0, s, A, lda, q, kp, Y, ldy, M,
                         N, K, kc, dnorm2, e_host, pp, ldp, nzr);
    else
      hipLaunchKernelGGL(sample_i8_kernel<256>, grid, dim3(512), 0, s, A, lda, q, kp, Y, ldy, M,
                         N, K, kc, dnorm2, e_host, pp, ldp, nzr);
  }
  QB_HIP_TRY(hipGetLastError());
  if (nzr > 1) {
    ProfScope ps(kKReduce, double(nzr) * M * N, 8.0 * (nzr + 1) * M * N, s);
    hipLaunchKernelGGL(i8_reduce_kernel, dim3(static_cast<unsigned>(cdiv(M * N, 256))), dim3(256),
                       0, s, part, nzr, ldp, Y, ldy, M, int64_t(N));
    QB_HIP_TRY(hipGetLastError());
  }
  return kOk;
}

}  // namespace qb
