// Kernel-level entry points for the test suite (declared in include/cbc_testing.h).
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/cbc.h"
#include "../../include/cbc_testing.h"
#include "cbc_internal.h"

using namespace cbc;

extern "C" int cbc_test_gemm(int M, int N, int K, const void* A, int a_c128, int transA, int conjA,
                             const void* B, int b_c128, int transB, int conjB, void* C, int c_c128,
                             int acc_fp64, int tile, void* stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return CBC_EINVAL;
  std::vector<int32_t> t(2 * (size_t)M + 2 * (size_t)N + 2 * (size_t)K);
  int32_t* am = t.data();
  int32_t* cm = am + M;
  int32_t* bn = cm + M;
  int32_t* cn = bn + N;
  int32_t* ak = cn + N;
  int32_t* bk = ak + K;
  for (int m = 0; m < M; ++m) { am[m] = transA ? m : m * K; cm[m] = m * N; }
  for (int n = 0; n < N; ++n) { bn[n] = transB ? n * K : n; cn[n] = n; }
  for (int k = 0; k < K; ++k) { ak[k] = transA ? k * M : k; bk[k] = transB ? k : k * N; }
  int32_t* d = nullptr;
  if (hipMalloc(&d, t.size() * sizeof(int32_t)) != hipSuccess) return CBC_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  int rc = CBC_OK;
  if (hipMemcpy(d, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
    rc = CBC_EHIP;
  } else {
    GemmArgs g;
    g.A = A; g.B = B; g.C = C; g.M = M; g.N = N; g.K = K;
    g.offAm = d; g.offCm = d + M; g.offBn = d + 2 * M; g.offCn = d + 2 * M + N;
    g.offAk = d + 2 * M + 2 * N; g.offBk = d + 2 * M + 2 * N + K;
    g.conjA = conjA; g.conjB = conjB;
    g.a_kfast = !transA; g.b_kfast = transB;
    g.alpha_dev = nullptr; g.alpha_dev2 = nullptr; g.alpha = 1.0;
    g.batch = 1; g.bsA = g.bsB = g.bsC = g.bsAlpha = g.bsAlpha2 = 0;
    g.mbase = 0;
    void* part = nullptr;
    if (tile == GEMM_AUTO) {
      // the compression's policy: split-K where it would split, the tile chosen at launch
      const int t1 = gemm_pick_tile(M, N, K, 1, acc_fp64 != 0);
      const int ks = gemm_pick_ksplit(M, N, K, 1, t1);
      if (ks > 1) {
        tile = t1;
        g.ksplit = ks;
        g.kchunk = ((K + ks - 1) / ks + 15) / 16 * 16;
        if (hipMalloc(&part, (size_t)ks * M * N * (acc_fp64 ? 16 : 8)) != hipSuccess) rc = CBC_ENOMEM;
        g.part = part;
      }
    }
    if (rc == CBC_OK &&
        launch_gemm(g, a_c128 ? DT_C128 : DT_C64, b_c128 ? DT_C128 : DT_C64,
                    c_c128 ? DT_C128 : DT_C64, acc_fp64 ? DT_C128 : DT_C64, tile, st) != hipSuccess)
      rc = CBC_EHIP;
    else if (rc == CBC_OK && hipStreamSynchronize(st) != hipSuccess)
      rc = CBC_EHIP;
    if (part) (void)hipFree(part);
  }
  (void)hipFree(d);
  return rc;
}

extern "C" int cbc_test_gemm_time(int M, int N, int K, int a_c128, int b_c128, int c_c128,
                                  int acc_fp64, int tile, int reps, float* ms) {
  if (M < 1 || N < 1 || K < 1 || reps < 1 || !ms) return CBC_EINVAL;
  std::vector<int32_t> t(2 * (size_t)M + 2 * (size_t)N + 2 * (size_t)K);
  int32_t* am = t.data();
  int32_t* cm = am + M;
  int32_t* bn = cm + M;
  int32_t* cn = bn + N;
  int32_t* ak = cn + N;
  int32_t* bk = ak + K;
  for (int m = 0; m < M; ++m) { am[m] = m * K; cm[m] = m * N; }
  for (int n = 0; n < N; ++n) { bn[n] = n; cn[n] = n; }
  for (int k = 0; k < K; ++k) { ak[k] = k; bk[k] = k * N; }
  const size_t ea = a_c128 ? 16 : 8, eb = b_c128 ? 16 : 8, ec = c_c128 ? 16 : 8;
  int32_t* d = nullptr;
  void *A = nullptr, *B = nullptr, *C = nullptr, *part = nullptr;
  int rc = CBC_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(&d, t.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&A, ea * M * K) != hipSuccess || hipMalloc(&B, eb * K * N) != hipSuccess ||
      hipMalloc(&C, ec * M * N) != hipSuccess) {
    rc = CBC_ENOMEM;
  } else if (hipMemcpy(d, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemset(A, 0, ea * M * K) != hipSuccess || hipMemset(B, 0, eb * K * N) != hipSuccess ||
             hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = CBC_EHIP;
  } else {
    GemmArgs g;
    g.A = A; g.B = B; g.C = C; g.M = M; g.N = N; g.K = K;
    g.offAm = d; g.offCm = d + M; g.offBn = d + 2 * M; g.offCn = d + 2 * M + N;
    g.offAk = d + 2 * M + 2 * N; g.offBk = d + 2 * M + 2 * N + K;
    g.conjA = 0; g.conjB = 0; g.a_kfast = 1; g.b_kfast = 0;
    g.alpha_dev = nullptr; g.alpha_dev2 = nullptr; g.alpha = 1.0;
    g.batch = 1; g.bsA = g.bsB = g.bsC = g.bsAlpha = g.bsAlpha2 = 0;
    g.mbase = 0;
    const DType ta = a_c128 ? DT_C128 : DT_C64, tb = b_c128 ? DT_C128 : DT_C64;
    const DType tc = c_c128 ? DT_C128 : DT_C64, tacc = acc_fp64 ? DT_C128 : DT_C64;
    if (tile == GEMM_AUTO) {
      const int t1 = gemm_pick_tile(M, N, K, 1, acc_fp64 != 0);
      const int ks = gemm_pick_ksplit(M, N, K, 1, t1);
      if (ks > 1) {
        tile = t1;
        g.ksplit = ks;
        g.kchunk = ((K + ks - 1) / ks + 15) / 16 * 16;
        if (hipMalloc(&part, (size_t)ks * M * N * (acc_fp64 ? 16 : 8)) != hipSuccess) rc = CBC_ENOMEM;
        g.part = part;
      }
    }
    if (rc == CBC_OK && launch_gemm(g, ta, tb, tc, tacc, tile, nullptr) != hipSuccess) rc = CBC_EHIP;
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && rc == CBC_OK; ++r)
      if (launch_gemm(g, ta, tb, tc, tacc, tile, nullptr) != hipSuccess) rc = CBC_EHIP;
    (void)hipEventRecord(e1, nullptr);
    if (rc == CBC_OK && hipEventSynchronize(e1) == hipSuccess) {
      float t_ms = 0.0f;
      (void)hipEventElapsedTime(&t_ms, e0, e1);
      *ms = t_ms / reps;
    } else {
      rc = CBC_EHIP;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  (void)hipFree(part);
  (void)hipFree(A);
  (void)hipFree(B);
  (void)hipFree(C);
  return rc;
}

extern "C" int cbc_test_eig_reduction(void* G, int s, int kmax, double tol, int reduction, void* U,
                                      void* lam, void* kkeep, void* inv_sqrt_l0, void* tstamp,
                                      void* stream);
extern "C" int cbc_test_eig(void* G, int s, int kmax, double tol, void* U, void* lam, void* kkeep,
                            void* inv_sqrt_l0, void* tstamp, void* stream) {
  return cbc_test_eig_reduction(G, s, kmax, tol, 0, U, lam, kkeep, inv_sqrt_l0, tstamp, stream);
}

extern "C" int cbc_test_eig_reduction(void* G, int s, int kmax, double tol, int reduction, void* U,
                                      void* lam, void* kkeep, void* inv_sqrt_l0, void* tstamp,
                                      void* stream) {
  if (reduction != 0 && reduction != 1) return CBC_EINVAL;
  if (!G || !U || !lam || !kkeep || !inv_sqrt_l0 || s < 1 || kmax < 1 || kmax > s) return CBC_EINVAL;
  double* w = nullptr;
  if (hipMalloc(&w, eig_work_doubles(s, kmax) * sizeof(double)) != hipSuccess) return CBC_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  EigArgs a;
  a.G = (double2*)G; a.s = s; a.kmax = kmax; a.tol = tol; a.U = (double2*)U;
  a.lam = (double*)lam; a.kkeep = (int*)kkeep; a.inv_sqrt_l0 = (double*)inv_sqrt_l0; a.work = w;
  a.tstamp = (long long*)tstamp;
  a.batch = 1;
  a.bs = 0;
  a.reduction = reduction;
  int rc = CBC_OK;
  if (launch_eig(a, st) != hipSuccess) rc = CBC_EHIP;
  else if (hipStreamSynchronize(st) != hipSuccess) rc = CBC_EHIP;
  (void)hipFree(w);
  return rc;
}

extern "C" int cbc_test_chol_inv(void* G, int k, double shift_rel, double drop_rel, void* Cinv,
                                 void* ndrop, void* tstamp, void* stream) {
  if (!G || !Cinv || !ndrop || k < 1) return CBC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  CholArgs a;
  a.G = (double2*)G; a.k = k; a.shift_rel = shift_rel; a.drop_rel = drop_rel;
  a.Cinv = (double2*)Cinv; a.log_scale = nullptr; a.scale = nullptr; a.ndrop = (int*)ndrop;
  a.tstamp = k <= CHOL_LDS_MAX ? (long long*)tstamp : nullptr;
  a.batch = 1;
  a.bs = 0;
  double2* w = nullptr;
  if (k > CHOL_LDS_MAX) {
    if (hipMalloc(&w, chol_work_doubles(k) * sizeof(double)) != hipSuccess) return CBC_ENOMEM;
    a.work = w;
  }
  int rc = CBC_OK;
  if (launch_chol_inv(a, st) != hipSuccess) rc = CBC_EHIP;
  else if (hipStreamSynchronize(st) != hipSuccess) rc = CBC_EHIP;
  if (w) (void)hipFree(w);
  return rc;
}

extern "C" int cbc_test_eig_report(void* G, int s, int kmax, double tol, int force_timeout,
                                   void* U, void* lam, void* kkeep, void* inv_sqrt_l0,
                                   void* status, void* rec, void* stream) {
  if (!G || !U || !lam || !kkeep || !inv_sqrt_l0 || !status || !rec || s < 1 || kmax < 1 ||
      kmax > s)
    return CBC_EINVAL;
  double* w = nullptr;
  if (hipMalloc(&w, eig_work_doubles(s, kmax) * sizeof(double)) != hipSuccess) return CBC_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  EigArgs a;
  a.G = (double2*)G; a.s = s; a.kmax = kmax; a.tol = tol; a.U = (double2*)U;
  a.lam = (double*)lam; a.kkeep = (int*)kkeep; a.inv_sqrt_l0 = (double*)inv_sqrt_l0; a.work = w;
  a.tstamp = nullptr;
  a.batch = 1;
  a.bs = 0;
  a.status = (int*)status;
  a.rec = (cbc_trunc_record*)rec;
  a.rec_node = 7;
  a.rec_sweep = 2;
  if (force_timeout) {
    // the time-out path exists only in the multi-workgroup reduction
    a.timeout_ticks = -1;
    a.reduction = 1;
  }
  int rc = CBC_OK;
  if (launch_eig(a, st) != hipSuccess) rc = CBC_EHIP;
  else if (hipStreamSynchronize(st) != hipSuccess) rc = CBC_EHIP;
  (void)hipFree(w);
  return rc;
}
