// Internal interfaces between the host planner/executor and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cbc.h"

namespace cbc {

// Element types used for operands.
enum DType : int { DT_C64 = 0, DT_C128 = 1 };

// Generic complex tensor-contraction GEMM:
//   C[m, n] = alpha * sum_k opA(A)[m, k] * opB(B)[k, n]
// where every row/column/reduction index is mapped to a complex-element offset through device
// tables (offAm[m] + offAk[k] addresses A, offBk[k] + offBn[n] addresses B, offCm[m] + offCn[n]
// addresses C). This covers any leg order of the operands without transposes.
struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  const int32_t* offAm;
  const int32_t* offAk;
  const int32_t* offBk;
  const int32_t* offBn;
  const int32_t* offCm;
  const int32_t* offCn;
  int conjA, conjB;
  int a_kfast;              // 1: consecutive k are adjacent in A; 0: consecutive m are
  int b_kfast;              // 1: consecutive k are adjacent in B; 0: consecutive n are
  const double* alpha_dev;  // optional device scalar multiplier (nullptr: none)
  const double* alpha_dev2; // optional second device scalar multiplier (nullptr: none)
  double alpha;             // host scalar multiplier
  // batch: instance z (blockIdx.z) uses every pointer advanced by z times its byte stride
  int batch;
  int64_t bsA, bsB, bsC, bsAlpha, bsAlpha2;
  int mbase = 0;   // first row of this launch (the launcher splits very tall problems into row chunks)
  // split-K: the reduction range is cut into ksplit chunks of kchunk (a multiple of 16); chunk z of
  // instance b writes its raw sums to part_b[(z * M + m) * N + n] (accumulator type, part_b = part +
  // b * bsPart bytes), and a second kernel adds the chunks in order and applies alpha and C offsets
  int ksplit = 1;
  int kchunk = 0;
  void* part = nullptr;
  int64_t bsPart = 0;   // per-instance byte stride of part
  // dense mode (offAm == nullptr): element offsets are m * sAm + k * sAk, k * sBk + n * sBn and
  // m * sCm + n * sCn instead of table lookups
  int64_t sAm = 0, sAk = 0, sBk = 0, sBn = 0, sCm = 0, sCn = 0;
  int accum = 0;        // 1: C += alpha * op(A) op(B)
  // 1: C is Hermitian by construction (B is the conjugate of A over relabelled legs, M == N): only
  // entries m >= n are computed, and each strictly lower one is also written, conjugated, at (n, m)
  int herm = 0;
  // optional device flag per instance (advancing by bsSkip bytes): the launch does nothing where it
  // is set (the blocked Cholesky's steps after an identity shortcut)
  const int* skip = nullptr;
  int64_t bsSkip = 0;
};
// pointer of instance b for a per-instance byte stride
template <typename T>
__host__ __device__ inline T* inst_ptr(T* p, int64_t stride, int b) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<void*>(
                 reinterpret_cast<const void*>(p))) + stride * (int64_t)b)
           : p;
}

// Tile configurations of the contraction GEMM: table-driven 32x32 / 64x64 tiles, the pipelined
// kernel with 64x64 tiles, or (FP32 accumulation only) the pipelined kernel with 128x128 tiles on
// eight waves; GEMM_AUTO picks by shape. Split-K works with the 32x32 and the pipelined tiles.
enum GemmTile : int { GEMM_AUTO = -1, GEMM_TILE32 = 0, GEMM_TILE64 = 1, GEMM_PIPE64 = 2, GEMM_PIPE128 = 3 };
int gemm_pick_tile(int M, int N, int K, int batch, bool fp64_acc);
// number of K chunks for a launch with too few output tiles for its tile size (1: no split)
int gemm_pick_ksplit(int M, int N, int K, int batch, int tile);
// Launch a GEMM. acc: DT_C64 -> FP32 MFMA, DT_C128 -> FP64 MFMA.
hipError_t launch_gemm(const GemmArgs& a, DType ta, DType tb, DType tc, DType acc, int tile,
                       hipStream_t s);

// Truncation eigensolve of a Hermitian FP64 Gram matrix G (s x s, row-major, both triangles valid,
// overwritten). Writes the top-kmax eigenvectors as columns of U (s x kmax, row-major, complex128),
// descending eigenvalues lam[0..kmax), the number kept (<= kmax, >= 1) to *kkeep, and
// 1/sqrt(lam[0]) to *inv_sqrt_l0. Columns of U beyond the kept count are zero.
struct EigArgs {
  double2* G;
  int s;
  int kmax;
  double tol;       // relative singular-value cutoff (0: keep kmax)
  double2* U;
  double* lam;
  int* kkeep;
  double* inv_sqrt_l0;
  double* work;     // scratch, eig_work_doubles(s, kmax) doubles
  long long* tstamp;  // optional: wall-clock stamps at phase boundaries (8 entries), or nullptr
  int batch;          // instances; every pointer above (except tstamp) advances by bs bytes
  int64_t bs;
  int spread = 1;     // set by launch_eig: grid widening of the XCD-aware launches (1 or 8)
  // optional (advance by bs like the pointers above): the call's device status word (a failure
  // code is stored there if it still holds 0) and the record of this truncation
  int* status = nullptr;
  cbc_trunc_record* rec = nullptr;
  int rec_node = -1, rec_sweep = 0;
  // wall-clock ticks (100 MHz) a cross-workgroup wait may take before the solve gives up; a
  // negative value makes the first wait give up at once (tests of the status path)
  long long timeout_ticks = 200000000LL;
  // reduction to tridiagonal form for s > 128: 0 = two-stage (dense -> band -> tridiagonal),
  // 1 = one-stage multi-workgroup (s <= 1536, see eig_pick_reduction)
  int reduction = 0;
};
size_t eig_work_doubles(int s, int kmax);
// largest Gram the eigensolver handles
bool eig_size_supported(int s);
// reduction for a solve of this size (EigArgs::reduction): 1 (one-stage, multi-workgroup) for a
// single instance outside a caller's stream capture where it applies, otherwise 0 (two-stage)
int eig_pick_reduction(int s, int batch, bool caller_capture);
// a solve of this size may take the multi-workgroup reduction, whose workgroups wait for each
// other (its eager launches and the graphs holding it are ordered device-wide)
bool eig_needs_gate(int s);
hipError_t launch_eig(const EigArgs& a, hipStream_t st);

// Device-wide order of the solves whose workgroups wait for each other: mw_gate_enter makes `st`
// wait for the previous such solve queued eagerly on the current device from another stream,
// mw_gate_leave records the one just queued. Both do nothing on a capturing stream.
hipError_t mw_gate_enter(hipStream_t st);
hipError_t mw_gate_leave(hipStream_t st);

// n-side truncation output: L[j, c] = sqrt(max(lam_j, 0)) / sqrt(lam_0) * conj(V[c, j]) for j < kkeep,
// zero for kkeep <= j < kmax. L is kmax x n, written in the contraction precision.
hipError_t launch_form_l_nside(const double2* V, const double* lam, const int* kkeep, int n,
                               int kmax, void* L, DType tl, int batch, int64_t bs, hipStream_t st);

// Cholesky of a Hermitian PSD Gram G (k x k, FP64, overwritten) with an optional diagonal shift of
// shift_rel * trace(G); pivots below drop_rel * max pivot are dropped. Writes Cinv = C^{-1} (k x k,
// lower triangular, zero rows/columns for dropped pivots) and, if log_scale != nullptr,
// log_scale[0] = -0.5 * log(trace(G)) and scale[0] = 1/sqrt(trace(G)).
struct CholArgs {
  double2* G;
  int k;
  double shift_rel;
  double drop_rel;
  double2* Cinv;
  double* log_scale;
  double* scale;
  int* ndrop;
  long long* tstamp;  // optional: wall-clock stamps at phase boundaries (4 entries), or nullptr
  int batch;          // instances; every pointer above (except tstamp) advances by bs bytes
  int64_t bs;
  double2* work = nullptr;   // k > CHOL_LDS_MAX: chol_work_doubles(k) doubles of scratch
  // internal (diagonal blocks of the blocked factorisation): row stride of G and Cinv, and an
  // absolute pivot threshold read from the device (the shift is then already applied)
  int ld = 0;
  const double* thresh_dev = nullptr;
  int* status = nullptr;   // optional device status word (CBC_ENOTPD on a non-finite Gram)
  const int* skip = nullptr;   // internal: device flag; the kernel does nothing where it is set
};
// largest k factorised by one LDS-resident workgroup; larger ones are blocked and need `work`
constexpr int CHOL_LDS_MAX = 88;
size_t chol_work_doubles(int k);
hipError_t launch_chol_inv(const CholArgs& a, hipStream_t st);

// Workspace of cbc_apply_noalloc: a static device array of this many bytes per GPU (noalloc.hip);
// noalloc_scratch gives its address on the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
hipError_t noalloc_scratch(void** ptr);

// Elementwise helpers.
// Batched elementwise helpers: instance b uses src + b * ss and dst + b * ds (bytes).
hipError_t launch_convert(const void* src, DType ts, void* dst, DType td, int64_t n, int batch,
                          int64_t ss, int64_t ds, hipStream_t st);
// x *= 1/||x||_F in place (n complex elements of type t, one instance); the factor to scale[0] and
// its logarithm to logs[0] if given; a non-finite norm stores CBC_ENOTPD in *status (if given).
// `part` is scratch of NORM_MAX_BLOCKS doubles (per-block partial sums, added in a fixed order).
constexpr int NORM_MAX_BLOCKS = 512;
int norm_blocks(int64_t n);
hipError_t launch_normalize(void* x, DType t, int64_t n, double* part, double* scale, double* logs,
                            int* status, hipStream_t st);
hipError_t launch_fill_identity(void* dst, DType t, int rows, int cols, int batch, int64_t ds,
                                hipStream_t st);
hipError_t launch_zero(void* dst, int64_t bytes, int batch, int64_t ds, hipStream_t st);
// Report header at the start of a call's workspace: 64 bytes holding magic, status 0, dropped
// pivots 0, the record count and the records' byte offset (int64 at byte 16); the n_rec records of
// rec_bytes each at rec_off are zeroed.
hipError_t launch_report_header(void* ws, uint32_t magic, int n_rec, int64_t rec_off,
                                int64_t rec_bytes, int batch, int64_t ds, hipStream_t st);
// Output writer: src is a (a x b x rest) tensor in type ts; writes dst[(b, a, rest)] as complex128
// (swap of the two leading legs), multiplied by exp(-sum(logs[0..nlogs))) if logs != nullptr.
hipError_t launch_write_out(const void* src, DType ts, int a, int b, int64_t rest, double2* dst,
                            const double* logs, int nlogs, int batch, int64_t ss, int64_t ds,
                            int64_t ls, hipStream_t st);

}  // namespace cbc
