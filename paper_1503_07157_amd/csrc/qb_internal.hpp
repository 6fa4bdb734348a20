// Internal declarations shared by the HIP translation units of the QB
// library.  Not part of the public C ABI (include/qb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <cstddef>
#include <cstdint>

namespace qb {

// ---- status codes (mirror include/qb.h) ----------------------------------
constexpr int kOk = 0;
constexpr int kEInval = -1;
constexpr int kENonfinite = -2;
constexpr int kEWorkspace = -3;
constexpr int kEHip = -4;
constexpr int kENoDevice = -5;

#define QB_HIP_TRY(expr)                                 \
  do {                                                   \
    hipError_t qb_err_ = (expr);                         \
    if (qb_err_ != hipSuccess) return ::qb::kEHip;       \
  } while (0)

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// waits for every outstanding global store of the thread, which a kernel
// that streams results to global memory between barriers does not need.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- GEMM tiling shared by the FP64 kernels ------------------------------
constexpr int kTileM = 128;      // workgroup output rows
constexpr int kTileN = 128;      // workgroup output columns
constexpr int kTileK = 16;       // reduction depth staged per LDS fill
constexpr int kGemmThreads = 256;
constexpr int kMaxSplit = 256;   // split-K partial buffers (upper bound)
constexpr int kNumCU = 256;                     // MI355X compute units
constexpr int64_t kSplitMinDepth = 128;         // smallest reduction depth per workgroup
constexpr int64_t kPartialCapDoubles = int64_t(16) << 20;  // 128 MiB of partials at most
constexpr int kMaxPanel = 256;   // widest block (b) supported by orth

// Leading dimensions and the row counts of panels stay below 2^24: the tile
// loads use 32-bit element offsets over up to 256 rows or columns.
constexpr int64_t kMaxLd = int64_t(1) << 24;
// The downdate grid puts the column tiles (64 wide) in grid.y.
constexpr int64_t kMaxDowndateCols = int64_t(65535) * 64;

// QB_ENODEVICE unless the current HIP device is a gfx950; the answer is
// cached per device, so only the first call on a device queries it.
int device_ready();

// roctx range for the duration of a scope (shown by rocprofv3 --marker-trace;
// a few nanoseconds when no tool listens)
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Workspace arena: bump allocator over a caller buffer, 256-byte aligned.
struct Arena {
  char* base;
  size_t cap;
  size_t used;
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    size_t bytes = count * sizeof(T);
    if (base == nullptr) { used = off + bytes; return nullptr; }  // sizing pass
    if (off + bytes > cap) { used = off + bytes; return nullptr; }
    used = off + bytes;
    return reinterpret_cast<T*>(base + off);
  }
};

// ---- optional per-kernel timing -------------------------------------------
// When enabled, every launch is bracketed by two HIP events on its stream
// and tagged with the algorithmic flops and bytes of the operation it
// performs.  Elapsed times are folded in when the counters are read.
enum KernelId {
  kKSketch = 0, kKGemmNN, kKGemmTN, kKReduce, kKDowndate, kKChol, kKTrinv, kKNorm, kKCopy,
  kKGemmNNLowp, kKGemmTNLowp, kKGemmNNSmall, kKGemmTNSmall, kKGemmNNTall,
  kKBatchSample, kKBatchGram, kKBatchApply, kKBatchReproj, kKBatchB, kKBatchDowndate,
  kKCholBatched, kKBatchMisc, kKSampleI8, kKCount
};
const char* kernel_name(int id);
bool prof_enabled();
// returns an opaque token (or -1 when profiling is off); call prof_end after the launch
int prof_begin(int id, double flops, double bytes, hipStream_t s);
void prof_end(int token, hipStream_t s);
struct ProfScope {
  int token;
  hipStream_t s;
  ProfScope(int id, double flops, double bytes, hipStream_t st)
      : token(prof_enabled() ? prof_begin(id, flops, bytes, st) : -1), s(st) {}
  ~ProfScope() { if (token >= 0) prof_end(token, s); }
};

// ---- kernel launchers (each returns a status code) ------------------------

// sketch columns [col0, col0 + w) -> out (n x w, ld)
int launch_sketch(uint64_t seed, int64_t n, int64_t col0, int w, double* out, int64_t ld,
                  hipStream_t s);

// split-K choice for an M x N product with reduction depth K (output tiles of
// kTileM x kTileN): enough workgroups to fill the chip, at least
// kSplitMinDepth per workgroup, partial storage bounded by kPartialCapDoubles
int choose_split(int64_t M, int64_t N, int64_t K, int slots_per_cu = 2, bool tall_nn = false);
// the split with the best-filled last round of workgroups, for output tiles
// of bm x bn
int choose_split_fill(int64_t M, int64_t N, int64_t K, int slots_per_cu, int bm = kTileM,
                      int bn = kTileN);
// split-K of the low-precision products (their own tile shapes and
// workgroups per CU): Y = X W (nn) or C = Q^T X
int lowp_split(int precision, bool nn, int64_t M, int64_t N, int64_t K);
// doubles of partial storage for an M x N product split `split` ways
size_t partial_doubles(int64_t M, int64_t N, int split);

// Y(M x N) = alpha * X(M x K, ldx) * W(K x N, ldw) + beta * Y, FP64.
// part: split-K partial buffer (partial_doubles(M, N, split) doubles) or
// nullptr when split == 1.
int gemm_nn(const double* X, int64_t ldx, const double* W, int64_t ldw, double* Y, int64_t ldy,
            int64_t M, int64_t N, int64_t K, double alpha, double beta, int split, double* part,
            hipStream_t s);

// C(P x N) = Q(K x P, ldq)^T * X(K x N, ldx), FP64; written to C (ldc) or,
// when transpose_out, C^T to an N x P matrix (ldc).  sq_part, if non-null,
// receives per-workgroup partial sums of squares of C (sq_count out).
int gemm_tn(const double* Qm, int64_t ldq, const double* X, int64_t ldx, double* C, int64_t ldc,
            int64_t P, int64_t N, int64_t K, bool transpose_out, int split, double* part,
            double* sq_part, int* sq_count, hipStream_t s);

// Exact-range sample Y = A~ Omega~ on the int8 MFMA (k_sample_i8.hip).
// quantize_sketch: Omega (n x w, ldo) -> int8 sketch q of sample_i8_kp(n) x w
// bytes (column-major, zero padded).  sample_i8: Y (M x N, N <= 256) from A
// (M x K, lda) and q; the exponent comes from the device scalar *dnorm2
// (||A||_F^2) or, when dnorm2 is null, from e_host.  part: split-K partials
// of sample_i8_partials(M, N, K) doubles.
int64_t sample_i8_kp(int64_t K);
int sample_i8_split(int64_t M, int64_t K);
size_t sample_i8_partials(int64_t M, int64_t N, int64_t K);
int quantize_sketch(const double* om, int64_t ldo, int64_t n, int w, int8_t* q, hipStream_t s);
int sample_i8(const double* A, int64_t lda, const int8_t* q, double* Y, int64_t ldy, int64_t M,
              int N, int64_t K, const double* dnorm2, int e_host, double* part, hipStream_t s);

// mixed-precision sampling variants (precision: 1 = f32, 2 = bf16x3):
// Y(M x N) = X W and C(P x N) = Q^T X (or C^T, transpose_out), with the
// panel (W, or Q) rounded once into scratch, followed there by the split-K
// partials: lowp_scratch_doubles(precision, nn, M, N, K) doubles (M = P for
// C = Q^T X), 256-byte aligned, required.
size_t lowp_scratch_doubles(int precision, bool nn, int64_t M, int64_t N, int64_t K);
int gemm_nn_lowp(int precision, const double* X, int64_t ldx, const double* W, int64_t ldw,
                 double* Y, int64_t ldy, int64_t M, int64_t N, int64_t K, int split,
                 double* scratch, hipStream_t s);
int gemm_tn_lowp(int precision, const double* Qm, int64_t ldq, const double* X, int64_t ldx,
                 double* C, int64_t ldc, int64_t P, int64_t N, int64_t K, bool transpose_out,
                 int split, double* scratch, hipStream_t s);

// R(M x N) -= Q(M x K) * B(K x N); per-workgroup sums of squares of the
// updated R into sq_part (count returned through sq_count).
int downdate(double* R, int64_t ldr, const double* Qm, int64_t ldq, const double* B, int64_t ldb,
             int64_t M, int64_t N, int64_t K, double* sq_part, int* sq_count, hipStream_t s);
size_t downdate_partials(int64_t M, int64_t N);

// per-workgroup sums of squares of X and a non-finite flag
int sumsq_partials(const double* X, int64_t ldx, int64_t M, int64_t N, double* sq_part,
                   int* sq_count, int* nonfinite, hipStream_t s);
size_t sumsq_partials_count(int64_t M, int64_t N);
// out[0] = compensated sum of part[0..count) (hi + lo)
int sum_partials(const double* part, int count, double* out, hipStream_t s);

// Y(M x N, ldy) = X(M x N, ldx)
int copy_matrix(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t M, int64_t N,
                hipStream_t s);
int zero_matrix(double* Y, int64_t ldy, int64_t M, int64_t N, hipStream_t s);

// ---- batched forms (many independent problems in one launch) -------------
// One problem of a batched product.  op NN: C(M x N) = alpha A(M x K) B(K x N)
// + beta C; op TN: C(M x N) = A(K x M)^T B(K x N) (sq: per-tile sums of
// squares of C, or null); op DD: C(M x N) -= A(M x K) B(K x N) with per-tile
// sums of squares of the updated C into sq.  Workgroups [tile0, tile0 +
// tiles_m * tiles_n * ksplit) of the launch belong to this problem; every
// problem of one launch has the launch's tile class.
struct BatchGemm {
  const double* A;
  const double* B;
  double* C;
  double* sq;
  double* part;    // split-K partial tiles, ksplit slots of (tiles_m bm) x (tiles_n bn)
  int64_t lda, ldb, ldc;
  int64_t tile0;   // first workgroup of this problem in the product launch
  int64_t rblock0; // first workgroup of this problem in the reduce launch
  int32_t M, N, K;
  int32_t tiles_m, tiles_n;
  int32_t ksplit, kchunk;  // depth split: ksplit chunks of kchunk (a multiple of kTileK)
  int32_t bm, bn;          // output tile of the launch this problem belongs to
  int32_t cls;             // its tile class (host bookkeeping)
  int32_t vec;  // A and B 16-byte aligned with even leading dimensions
  double alpha, beta;
};
enum { kBatchNN = 0, kBatchTN = 1, kBatchDD = 2 };
constexpr int kBatchTile = 64;      // the default (and downdate) tile of batched products
// tile classes of batched products: 64 x 64; 16 x 16 / 32 x 32 for the
// Gram matrices of narrow panels; 64 x 32 / 32 x 64 for the other products
// of panels at most 32 wide (narrow N / narrow M)
enum { kTile64 = 0, kTileG16, kTileG32, kTileN32, kTileM32, kTileClasses };
void batch_tile_dims(int cls, int* bm, int* bn);
// the same dimensions for device code (checked against the kernels' shapes
// in k_gemm_batched.hip)
__host__ __device__ inline void batch_tile_dims_hd(int cls, int* bm, int* bn) {
  switch (cls) {
    case kTileG16: *bm = 16; *bn = 16; return;
    case kTileG32: *bm = 32; *bn = 32; return;
    case kTileN32: *bm = 64; *bn = 32; return;
    case kTileM32: *bm = 32; *bn = 64; return;
    default: *bm = kBatchTile; *bn = kBatchTile; return;
  }
}
constexpr int kBatchRed = 1024;     // elements per workgroup of the split-K reduction
// prof_id, flops, bytes: the profiler entry and the launch's algorithmic
// flops (sum of 2 M N K) and bytes (sum of 8 (M K + K N + M N), M N twice
// when C is also read).
// Units are (problem, tile, depth chunk) triples.  Problems with
// ksplit > 1 leave C to gemm_batched_reduce, which sums their chunks in
// order (alpha sum + beta C for NN, the sum for TN) with per-workgroup sums
// of squares into sq when sq is set; total_rblocks counts its workgroups.
// dev_total: the device count of the launch's units, planned on the device;
// total_tiles (total_rblocks) is an upper bound on it from the host (the
// captured launch keeps its grid while the work shrinks).  Bounds up to 2^22
// launch one workgroup per unit, the ones past the device count exiting at
// once; larger bounds launch a fixed grid that takes units from dev_next,
// the launch's unit counter (zeroed before the launch).  Both are required.
int gemm_batched(int op, int cls, const BatchGemm* desc, int count, int64_t total_tiles,
                 int prof_id, double flops, double bytes, hipStream_t s,
                 const int64_t* dev_total, unsigned long long* dev_next);
int gemm_batched_reduce(int op, const BatchGemm* desc, int count, int64_t total_rblocks,
                        int prof_id, hipStream_t s, const int64_t* dev_total,
                        unsigned long long* dev_next);

struct BatchChol {  // Cholesky with dropping + inverse of one w x w Gram matrix
  const double* G;    // G (ld w), unless part is set
  int* kept;
  double* Tinv;
  int32_t w;
  int32_t ksplit;     // > 1: G is the sum of the Gram product's depth chunks
  const double* part; // chunk z at part + z slot, element (i, j) at i + j ldp
  int64_t ldp, slot;
};
int chol_inv_batched(const BatchChol* desc, int count, hipStream_t s);  // w <= 64

struct BatchSketch {  // columns [col0, col0 + w) of the n x inf sketch of seed
  uint64_t seed;
  int64_t n, col0, ld;
  double* out;
  int64_t block0;
  int32_t w;
};
// dev_total: the device count of units, walked in strides of the grid
int sketch_batched(const BatchSketch* desc, int count, int64_t total_blocks, hipStream_t s,
                   const int64_t* dev_total);
int64_t sketch_blocks(int64_t n, int w);

struct BatchConvert {  // R = double(A) (A float, m x n) with sums of squares and
  const float* A;      // non-finite flags per workgroup
  double* R;
  double* part;
  int* flags;
  int64_t lda, ldr, m, n;
  int64_t block0;
};
int convert_batched(const BatchConvert* desc, int count, int64_t total_blocks, hipStream_t s);
int64_t convert_blocks(int64_t m, int64_t n);

struct BatchSum {  // out[0..1] = compensated sum of part[0..count) (hi, lo);
  const double* part;  // iflag = OR of flags[0..count) when flags is set
  const int* flags;
  double* out;
  int* iflag;
  int32_t count;
};
int sum_batched(const BatchSum* desc, int count, hipStream_t s);

// orth: CholQR2 with dropping.  X (m x w, ldx) -> Q (m x w, ldq), kept
// columns first, zero columns after; *kept_dev receives the count.
struct OrthWork {
  double* gram;      // w x w
  double* tfull;     // w x w
  double* tinv;      // w x w
  double* qtmp;      // m x w (ld = ldt)
  int64_t ldt;
  int* kept;         // device: [0] count, [1..w] kept indices
  double* part;      // split-K partials for the Gram
  int split;
};
size_t orth_work_bytes(int64_t m, int w);
int orth_carve(Arena& a, int64_t m, int w, OrthWork* ow);
int orth_cholqr2(const double* X, int64_t ldx, double* Q, int64_t ldq, int64_t m, int w,
                 const OrthWork& ow, hipStream_t s);
// orth_cholqr2 that also returns R^{-1} (w x w, ld w) of X = Q R, with
// R = T2 T1 the product of the two passes' factors (t1inv: w x w scratch),
// and sets *dropped (device int) to 1 when either pass dropped a column
int orth_cholqr2_rinv(const double* X, int64_t ldx, double* Q, int64_t ldq, int64_t m, int w,
                      const OrthWork& ow, double* t1inv, double* rinv, int* dropped,
                      hipStream_t s);

}  // namespace qb
