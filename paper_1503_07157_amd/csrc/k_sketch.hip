// Gaussian sketch Omega (Figure 4 step (2), Figure 6 step (2); Section 4.1
// eq. (OmegaBlock)): entry (i, j) of an n x infinity Gaussian matrix is a
// pure function of (seed, i, j).  Rows 2t and 2t+1 of column j come from one
// Philox4x32-10 evaluation (Salmon et al., SC'11) of counter (t, j, 0, 0)
// under key (seed_lo, seed_hi), turned into two normals by Box-Muller.
//
// The transform uses only correctly rounded IEEE double operations in a
// fixed order (this file is built with floating-point contraction off), so
// the result is reproducible bit for bit by any IEEE double implementation
// of the same steps:
//   u1 = ((x0 << 21 | x1 >> 11) + 1) 2^-53,  u2 likewise from (x2, x3)
//   log u1: u1 = f 2^e, f in [sqrt(1/2), sqrt(2)), s = (f - 1)/(f + 1),
//           log f = 2 s sum_{k=0}^{10} s^{2k}/(2k+1)  (atanh series),
//           log u1 = e ln2_hi + (log f + e ln2_lo)
//   cos/sin(2 pi u2): x = 4 u2, q = rint(x), phi = (x - q) pi/2, Taylor
//           series (sin to phi^17, cos to phi^18), quarter-turn rotation by q
//   Omega(2t, j) = rho cos, Omega(2t+1, j) = rho sin, rho = sqrt(-2 log u1)
#include "qb_internal.hpp"

#pragma clang fp contract(off)

namespace qb {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;  // Philox4x32 multipliers
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;     // key increments (golden ratio, sqrt(3)-1)
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

// ln 2 split: hi = nearest double to ln 2 with the low 20 significand bits
// cleared (33 significant bits, so e * hi is exact for |e| < 2^20);
// lo = nearest double to (ln 2 - hi).
constexpr double kLn2Hi = 0x1.62e42fef00000p-1;
constexpr double kLn2Lo = 0x1.473de6af278edp-34;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;  // nearest double to sqrt(1/2)
constexpr double kHalfPi = 0x1.921fb54442d18p+0;    // nearest double to pi/2

struct Words { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += kWeyl0; k1 += kWeyl1; }
    const uint32_t hi0 = __umulhi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint32_t hi1 = __umulhi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  const uint64_t v = ((static_cast<uint64_t>(hi) << 21) | (lo >> 11)) + 1ull;
  return static_cast<double>(v) * 0x1p-53;
}

// natural log for normal u in (0, 1]
__device__ __forceinline__ double log_fixed(double u) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(u));
  int e = static_cast<int>((bits >> 52) & 0x7ffu) - 1022;
  double f = __longlong_as_double(static_cast<long long>((bits & 0x000FFFFFFFFFFFFFull) |
                                                         0x3FE0000000000000ull));
  if (f < kSqrtHalf) { f = f * 2.0; e -= 1; }
  const double s = (f - 1.0) / (f + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0;
  const double logf = (s + s) * p;
  const double ed = static_cast<double>(e);
  return ed * kLn2Hi + (logf + ed * kLn2Lo);
}

__device__ __forceinline__ void sincos_2pi_fixed(double u, double* cs, double* sn) {
  const double x = u * 4.0;
  const double q = rint(x);
  const double r = x - q;
  const double phi = r * kHalfPi;
  const double z = phi * phi;
  double ps = 1.0 / 355687428096000.0;          // 1/17!
  ps = ps * z + -1.0 / 1307674368000.0;         // -1/15!
  ps = ps * z + 1.0 / 6227020800.0;             // 1/13!
  ps = ps * z + -1.0 / 39916800.0;              // -1/11!
  ps = ps * z + 1.0 / 362880.0;                 // 1/9!
  ps = ps * z + -1.0 / 5040.0;                  // -1/7!
  ps = ps * z + 1.0 / 120.0;                    // 1/5!
  ps = ps * z + -1.0 / 6.0;                     // -1/3!
  ps = ps * z + 1.0;
  const double s = phi * ps;
  double pc = -1.0 / 6402373705728000.0;        // -1/18!
  pc = pc * z + 1.0 / 20922789888000.0;         // 1/16!
  pc = pc * z + -1.0 / 87178291200.0;           // -1/14!
  pc = pc * z + 1.0 / 479001600.0;              // 1/12!
  pc = pc * z + -1.0 / 3628800.0;               // -1/10!
  pc = pc * z + 1.0 / 40320.0;                  // 1/8!
  pc = pc * z + -1.0 / 720.0;                   // -1/6!
  pc = pc * z + 1.0 / 24.0;                     // 1/4!
  pc = pc * z + -1.0 / 2.0;                     // -1/2!
  pc = pc * z + 1.0;
  const double c = pc;
  switch (static_cast<int>(q) & 3) {
    case 0: *cs = c; *sn = s; break;
    case 1: *cs = -s; *sn = c; break;
    case 2: *cs = -c; *sn = -s; break;
    default: *cs = s; *sn = -c; break;
  }
}

// entries (2t, jj) and (2t + 1, jj) of columns [col0, col0 + w) of the sketch
__device__ __forceinline__ void sketch_pair(uint32_t k0, uint32_t k1, int64_t n, int64_t col0,
                                            double* __restrict__ out, int64_t ld, int64_t t,
                                            int64_t jj) {
  const uint32_t j = static_cast<uint32_t>(col0 + jj);
  const Words x = philox4x32_10(static_cast<uint32_t>(t), j, 0u, 0u, k0, k1);
  const double u1 = unit53(x.x0, x.x1);
  const double u2 = unit53(x.x2, x.x3);
  const double rho = sqrt(-2.0 * log_fixed(u1));
  double c, s;
  sincos_2pi_fixed(u2, &c, &s);
  double* col = out + jj * ld;
  col[2 * t] = rho * c;
  if (2 * t + 1 < n) col[2 * t + 1] = rho * s;
}

// one thread per (row pair t, column jj)
__global__ __launch_bounds__(256) void sketch_kernel(uint32_t k0, uint32_t k1, int64_t n,
                                                     int64_t col0, double* __restrict__ out,
                                                     int64_t ld) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t npairs = (n + 1) / 2;
  if (t >= npairs) return;
  sketch_pair(k0, k1, n, col0, out, ld, t, blockIdx.y);
}

// batch: workgroup -> (problem, pair block, column)
__device__ __forceinline__ void sketch_batched_unit(const BatchSketch* __restrict__ desc,
                                                    int count, int64_t blk) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].block0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  const BatchSketch d = desc[lo];
  const int64_t npairs = (d.n + 1) / 2;
  const int64_t nb = (npairs + 255) / 256;
  const int64_t lb = blk - d.block0;
  const int64_t t = (lb % nb) * 256 + threadIdx.x;
  if (t >= npairs) return;
  sketch_pair(static_cast<uint32_t>(d.seed), static_cast<uint32_t>(d.seed >> 32), d.n, d.col0,
              d.out, d.ld, t, lb / nb);
}

// total: the device unit count, walked in strides of the grid
__global__ __launch_bounds__(256) void sketch_batched_kernel(const BatchSketch* __restrict__ desc,
                                                             int count,
                                                             const int64_t* __restrict__ total) {
  const int64_t n = *total;
  for (int64_t blk = blockIdx.x; blk < n; blk += gridDim.x) sketch_batched_unit(desc, count, blk);
}

}  // namespace

int64_t sketch_blocks(int64_t n, int w) { return ((n + 1) / 2 + 255) / 256 * w; }

int sketch_batched(const BatchSketch* desc, int count, int64_t total_blocks, hipStream_t s,
                   const int64_t* dev_total) {
  if (count <= 0 || total_blocks <= 0) return kOk;
  if (total_blocks > INT32_MAX || dev_total == nullptr) return kEInval;  // one-dimensional grid
  ProfScope ps(kKSketch, 0.0, 0.0, s);
  hipLaunchKernelGGL(sketch_batched_kernel, dim3(static_cast<unsigned>(total_blocks)), dim3(256),
                     0, s, desc, count, dev_total);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int launch_sketch(uint64_t seed, int64_t n, int64_t col0, int w, double* out, int64_t ld,
                  hipStream_t s) {
  if (n <= 0 || w <= 0) return kOk;
  const int64_t npairs = (n + 1) / 2;
  dim3 grid(static_cast<unsigned>((npairs + 255) / 256), static_cast<unsigned>(w));
  ProfScope ps(kKSketch, 0.0, 8.0 * n * w, s);
  hipLaunchKernelGGL(sketch_kernel, grid, dim3(256), 0, s, static_cast<uint32_t>(seed),
                     static_cast<uint32_t>(seed >> 32), n, col0, out, ld);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

}  // namespace qb
