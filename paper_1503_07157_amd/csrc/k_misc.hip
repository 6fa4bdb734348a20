// Frobenius-norm reductions, the non-finite check on the input, and the
// copy / fill kernels of the QB driver.
//
// ||X||_F^2 (Section 2.1 notation) is formed as per-workgroup partial sums
// in a fixed order followed by one workgroup that adds the partials in
// double-double arithmetic (Knuth's two-sum), so the result is reproducible
// and accurate to about one rounding of the exact sum of the partials.
#include "qb_internal.hpp"

namespace qb {
namespace {

constexpr int kSumThreads = 256;
constexpr int kSumBlocksMax = 4096;

// s + e = a + b exactly (Knuth); an overflowed sum keeps s = inf, e = 0
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = isfinite(s) ? (a - (s - bb)) + (b - bb) : 0.0;
}

// grid-stride over the elements of X (column-major), per-block partials
__global__ __launch_bounds__(kSumThreads) void sumsq_kernel(const double* __restrict__ X,
                                                            int64_t ldx, int64_t M, int64_t N,
                                                            double* __restrict__ part,
                                                            int* __restrict__ flags) {
  __shared__ double red[kSumThreads / 64];
  __shared__ int fred[kSumThreads / 64];
  const int64_t total = M * N;
  double s = 0.0;
  int bad = 0;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = idx % M, j = idx / M;
    const double v = X[i + j * ldx];
    bad |= !isfinite(v);
    s += v * v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    bad |= __shfl_xor(bad, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[wave] = s; fred[wave] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    int f = 0;
    for (int w = 0; w < kSumThreads / 64; ++w) { t += red[w]; f |= fred[w]; }
    part[blockIdx.x] = t;
    if (flags) flags[blockIdx.x] = f;
  }
}

// one workgroup of NT threads: out[0] = hi, out[1] = lo of the sum of
// part[0..count); iflag[0] = OR of flags[0..count) when flags is non-null
template <int NT>
__device__ __forceinline__ void sum_partials_body(const double* __restrict__ part, int count,
                                                  const int* __restrict__ flags,
                                                  double* __restrict__ out,
                                                  int* __restrict__ iflag) {
  __shared__ double hs[NT], ls[NT];
  __shared__ int fs[NT];
  double hi = 0.0, lo = 0.0;
  int f = 0;
  // unrolled so that the loads issue ahead of the compensated sums (whose
  // order, and so the result, is unchanged)
#pragma unroll 8
  for (int i = threadIdx.x; i < count; i += NT) {
    double s, e;
    two_sum(hi, part[i], s, e);
    hi = s;
    lo += e;
    if (flags) f |= flags[i];
  }
  hs[threadIdx.x] = hi;
  ls[threadIdx.x] = lo;
  fs[threadIdx.x] = f;
  __syncthreads();
  for (int stride = NT / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) {
      double s, e;
      two_sum(hs[threadIdx.x], hs[threadIdx.x + stride], s, e);
      hs[threadIdx.x] = s;
      ls[threadIdx.x] = ls[threadIdx.x] + ls[threadIdx.x + stride] + e;
      fs[threadIdx.x] |= fs[threadIdx.x + stride];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double s, e;
    two_sum(hs[0], ls[0], s, e);
    out[0] = s;
    out[1] = e;
    if (iflag) iflag[0] = fs[0];
  }
}

// the per-tile sums of one factorisation (up to 25k for a 10^4 x 10^4
// downdate) take a wide workgroup
constexpr int kPartialSumThreads = 1024;

__global__ __launch_bounds__(kPartialSumThreads) void sum_partials_kernel(
    const double* __restrict__ part, int count, const int* __restrict__ flags,
    double* __restrict__ out, int* __restrict__ iflag) {
  sum_partials_body<kPartialSumThreads>(part, count, flags, out, iflag);
}

// one workgroup per problem of a batch
__global__ __launch_bounds__(kSumThreads) void sum_batched_kernel(const BatchSum* __restrict__ d) {
  const BatchSum b = d[blockIdx.x];
  if (b.count <= 0) return;  // a problem that takes no part in this step
  sum_partials_body<kSumThreads>(b.part, b.count, b.flags, b.out, b.iflag);
}

constexpr int kConvPer = 8;  // elements per thread in convert_batched_kernel

// R = double(A) for a batch of float matrices; per-workgroup sums of
// squares (of the converted values) and non-finite flags
__global__ __launch_bounds__(kSumThreads) void convert_batched_kernel(
    const BatchConvert* __restrict__ desc, int count) {
  __shared__ double red[kSumThreads / 64];
  __shared__ int fred[kSumThreads / 64];
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].block0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  const BatchConvert c = desc[lo];
  const int64_t lb = blk - c.block0;
  const int64_t total = c.m * c.n;
  double s = 0.0;
  int bad = 0;
#pragma unroll
  for (int q = 0; q < kConvPer; ++q) {
    const int64_t e = (lb * kConvPer + q) * kSumThreads + threadIdx.x;
    if (e < total) {
      const int64_t i = e % c.m, j = e / c.m;
      const double v = static_cast<double>(c.A[i + j * c.lda]);
      c.R[i + j * c.ldr] = v;
      bad |= !isfinite(v);
      s += v * v;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    bad |= __shfl_xor(bad, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[wave] = s; fred[wave] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    int f = 0;
    for (int w = 0; w < kSumThreads / 64; ++w) { t += red[w]; f |= fred[w]; }
    c.part[lb] = t;
    c.flags[lb] = f;
  }
}

__global__ __launch_bounds__(256) void copy_kernel(const double* __restrict__ X, int64_t ldx,
                                                   double* __restrict__ Y, int64_t ldy, int64_t M,
                                                   int64_t N) {
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < M;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
      Y[i + j * ldy] = X[i + j * ldx];
  }
}

__global__ __launch_bounds__(256) void zero_kernel(double* __restrict__ Y, int64_t ldy, int64_t M,
                                                   int64_t N) {
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < M;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
      Y[i + j * ldy] = 0.0;
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t sumsq_partials_count(int64_t M, int64_t N) {
  const int64_t total = M * N;
  int64_t nb = cdiv(total, kSumThreads * 8);
  if (nb > kSumBlocksMax) nb = kSumBlocksMax;
  if (nb < 1) nb = 1;
  return static_cast<size_t>(nb);
}

int sumsq_partials(const double* X, int64_t ldx, int64_t M, int64_t N, double* sq_part,
                   int* sq_count, int* nonfinite, hipStream_t s) {
  const unsigned nb = static_cast<unsigned>(sumsq_partials_count(M, N));
  {
    ProfScope ps(kKNorm, 2.0 * M * N, 8.0 * M * N, s);
    hipLaunchKernelGGL(sumsq_kernel, dim3(nb), dim3(kSumThreads), 0, s, X, ldx, M, N, sq_part,
                       nonfinite);
  }
  QB_HIP_TRY(hipGetLastError());
  if (sq_count) *sq_count = static_cast<int>(nb);
  return kOk;
}

// out[0..1] = (hi, lo); when flags != nullptr, out_flag[0] = OR of flags
int sum_partials_ex(const double* part, int count, const int* flags, double* out, int* out_flag,
                    hipStream_t s) {
  {
    ProfScope ps(kKNorm, double(count), 8.0 * count, s);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kPartialSumThreads), 0, s, part, count,
                       flags, out, out_flag);
  }
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int64_t convert_blocks(int64_t m, int64_t n) {
  return cdiv(m * n, static_cast<int64_t>(kSumThreads) * kConvPer);
}

int convert_batched(const BatchConvert* desc, int count, int64_t total_blocks, hipStream_t s) {
  if (count <= 0 || total_blocks <= 0) return kOk;
  if (total_blocks > INT32_MAX) return kEInval;  // one-dimensional grid
  ProfScope ps(kKBatchMisc, 0.0, 0.0, s);
  hipLaunchKernelGGL(convert_batched_kernel, dim3(static_cast<unsigned>(total_blocks)),
                     dim3(kSumThreads), 0, s, desc, count);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int sum_batched(const BatchSum* desc, int count, hipStream_t s) {
  if (count <= 0) return kOk;
  ProfScope ps(kKBatchMisc, 0.0, 0.0, s);
  hipLaunchKernelGGL(sum_batched_kernel, dim3(static_cast<unsigned>(count)), dim3(kSumThreads), 0,
                     s, desc);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int sum_partials(const double* part, int count, double* out, hipStream_t s) {
  return sum_partials_ex(part, count, nullptr, out, nullptr, s);
}

int copy_matrix(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t M, int64_t N,
                hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  dim3 grid(static_cast<unsigned>(cdiv(M, 256) < 64 ? cdiv(M, 256) : 64),
            static_cast<unsigned>(N < 4096 ? N : 4096));
  {
    ProfScope ps(kKCopy, 0.0, 16.0 * M * N, s);
    hipLaunchKernelGGL(copy_kernel, grid, dim3(256), 0, s, X, ldx, Y, ldy, M, N);
  }
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

int zero_matrix(double* Y, int64_t ldy, int64_t M, int64_t N, hipStream_t s) {
  if (M <= 0 || N <= 0) return kOk;
  dim3 grid(static_cast<unsigned>(cdiv(M, 256) < 64 ? cdiv(M, 256) : 64),
            static_cast<unsigned>(N < 4096 ? N : 4096));
  hipLaunchKernelGGL(zero_kernel, grid, dim3(256), 0, s, Y, ldy, M, N);
  QB_HIP_TRY(hipGetLastError());
  return kOk;
}

}  // namespace qb
