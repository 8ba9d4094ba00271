// FP64 Cholesky factorisation and triangular inverse for the QR on the parent leg.
//
// The QR of S on its parent leg (Sec. III A, Eq. tt_cbc_qr_decomp; Sec. III B, Eq. cbc_tree_qr) is
// computed as Cholesky-QR on the Gram matrix G = S S^H: G = C C^H, Q = C^{-1} S has orthonormal rows
// spanning the row space of S. The first pass adds a diagonal shift proportional to trace(G) so the
// factorisation exists for rank-deficient S; later passes re-orthogonalise without a shift.
// Pivots below drop_rel times the largest diagonal are dropped: their row and column of C^{-1} are
// zero, so the matching rows of Q vanish (they carried no weight of S).
//
// A re-orthogonalisation pass (no shift) whose Gram equals the identity to rounding writes the
// identity: its Cholesky factor and inverse are the identity to the same rounding.
#include <float.h>

#include <algorithm>

#include "cbc_internal.h"
#include "device_status.h"

namespace cbc {

static constexpr int CHOL_THREADS = 1024;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline CholArgs chol_inst(const CholArgs& a0, int b) {
  CholArgs a = a0;
  a.G = inst_ptr(a0.G, a0.bs, b);
  a.Cinv = inst_ptr(a0.Cinv, a0.bs, b);
  a.log_scale = inst_ptr(a0.log_scale, a0.bs, b);
  a.scale = inst_ptr(a0.scale, a0.bs, b);
  a.ndrop = inst_ptr(a0.ndrop, a0.bs, b);
  a.work = inst_ptr(a0.work, a0.bs, b);
  a.thresh_dev = inst_ptr(a0.thresh_dev, a0.bs, b);
  a.status = inst_ptr(a0.status, a0.bs, b);
  a.skip = inst_ptr(a0.skip, a0.bs, b);
  return a;
}

// LDS-resident variant for k <= CHOL_LDS_MAX, blocked by NBc = 8 columns.
//   factor:  for each panel, wave 0 factors the 8 panel columns with the panel rows in registers
//            (one row per lane, two for panels taller than 64 rows, so k <= 128), then all waves
//            apply the rank-8 update to the trailing lower triangle (two barriers per panel);
//   inverse: the columns of the 8x8 diagonal blocks of X = C^{-1} are formed in parallel (one lane
//            each), then block-row i of X is X_ij = -X_ii sum_{l=j}^{i-1} C_il X_lj (two barriers per
//            block-row).
// The factor lives in the lower triangle of M (row stride k+1, so column-wise lane accesses fall in
// distinct banks); X's strictly lower part is stored transposed in the upper triangle, its diagonal
// in xd.
static constexpr int NBc = 8;

// a double from lane `l` (uniform) of the wave
__device__ __forceinline__ double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

static_assert(CHOL_LDS_MAX <= 128, "the register panel holds two rows per lane");

// Factor panel columns p..pe-1 (rows p..k-1) by one wave: lane l holds row p + l and, with TWO
// (a panel taller than 64 rows), row p + l + 64 in registers; the pivot and the panel's
// diagonal-block entries are broadcast from their lanes. Entries above the diagonal are updated too
// but never read or stored.
template <bool TWO>
__device__ inline void chol_panel(double2* M, int ld, int k, int p, int pe, double thresh,
                                  int* dropped, int lane) {
  const int i0r = p + lane, i1r = p + 64 + lane;
  double2 R0[NBc], R1[NBc];
#pragma unroll
  for (int q = 0; q < NBc; ++q) {
    const bool inp = p + q < pe;
    R0[q] = inp && i0r < k ? M[i0r * ld + p + q] : make_double2(0.0, 0.0);
    if (TWO) R1[q] = inp && i1r < k ? M[i1r * ld + p + q] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int q = 0; q < NBc; ++q) {
    const int jj = p + q;
    if (jj >= pe) break;
    const double djj = readlane_d(R0[q].x, q);
    if (!(djj > thresh)) {
      R0[q] = make_double2(0.0, 0.0);
      if (TWO) R1[q] = make_double2(0.0, 0.0);
      if (lane == 0) dropped[jj] = 1;
      continue;
    }
    const double ic = rsqrt(djj);
    R0[q] = i0r == jj ? make_double2(djj * ic, 0.0) : make_double2(R0[q].x * ic, R0[q].y * ic);
    if (TWO) R1[q] = make_double2(R1[q].x * ic, R1[q].y * ic);
#pragma unroll
    for (int l = q + 1; l < NBc; ++l) {
      if (p + l >= pe) break;
      const double2 clj = make_double2(readlane_d(R0[q].x, l), readlane_d(R0[q].y, l));
      R0[l].x = fma(-R0[q].x, clj.x, R0[l].x);
      R0[l].x = fma(-R0[q].y, clj.y, R0[l].x);
      R0[l].y = fma(-R0[q].y, clj.x, R0[l].y);
      R0[l].y = fma(R0[q].x, clj.y, R0[l].y);
      if (TWO) {
        R1[l].x = fma(-R1[q].x, clj.x, R1[l].x);
        R1[l].x = fma(-R1[q].y, clj.y, R1[l].x);
        R1[l].y = fma(-R1[q].y, clj.x, R1[l].y);
        R1[l].y = fma(R1[q].x, clj.y, R1[l].y);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NBc; ++q) {
    if (p + q < pe) {
      if (i0r < k && i0r >= p + q) M[i0r * ld + p + q] = R0[q];
      if (TWO && i1r < k) M[i1r * ld + p + q] = R1[q];
    }
  }
}


__global__ __launch_bounds__(CHOL_THREADS) void k_chol_inv_lds(CholArgs a0) {
  const CholArgs a = chol_inst(a0, blockIdx.x);
  if (a.skip && *a.skip) return;
  extern __shared__ double2 M[];
  __shared__ double red[32];
  __shared__ double sh_thresh;
  const int k = a.k;
  const int ld = k + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  double* xd = reinterpret_cast<double*>(M + (size_t)k * ld);
  int* dropped = reinterpret_cast<int*>(xd + k);
  double2* T = reinterpret_cast<double2*>(dropped + ((k + 3) & ~3));   // k x NBc block-row scratch
  const int gld = a.ld > 0 ? a.ld : k;   // row stride of G and Cinv in global memory
  if (a.tstamp && tid == 0) a.tstamp[0] = wall_clock64();
  for (int i = tid; i < k * k; i += blockDim.x) M[(i / k) * ld + (i % k)] = a.G[(size_t)(i / k) * gld + (i % k)];
  for (int i = tid; i < k; i += blockDim.x) dropped[i] = 0;
  __syncthreads();
  if (!a.thresh_dev && a.shift_rel == 0.0) {
    // a re-orthogonalisation pass whose Gram is the identity to rounding (|G - I| <= 4 k u): its
    // Cholesky factor and inverse are the identity to rounding as well, so write that and stop
    double dev = 0.0;
    for (int i = tid; i < k * k; i += blockDim.x) {
      const int r = i / k, c = i % k;
      const double2 g = M[r * ld + c];
      dev = fmax(dev, fmax(fabs(g.x - (r == c ? 1.0 : 0.0)), fabs(g.y)));
    }
    dev = wmax(dev);
    if (lane == 0) red[wave] = dev;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < nwave; ++w) m = fmax(m, red[w]);
    if (m <= 4.0 * k * DBL_EPSILON * 0.5) {
      for (int idx = tid; idx < k * k; idx += blockDim.x) {
        const int i = idx / k, c = idx % k;
        a.Cinv[(size_t)i * gld + c] = make_double2(i == c ? 1.0 : 0.0, 0.0);
      }
      if (a.tstamp && tid == 0) a.tstamp[1] = a.tstamp[2] = a.tstamp[3] = wall_clock64();
      return;
    }
    __syncthreads();
  }
  if (a.thresh_dev) {
    // diagonal block of the blocked factorisation: shift applied, threshold given
    if (tid == 0) sh_thresh = a.thresh_dev[0];
  } else {
  double tr = 0.0;
  for (int i = tid; i < k; i += blockDim.x) tr += M[i * ld + i].x;
  tr = wsum(tr);
  if (lane == 0) red[wave] = tr;
  __syncthreads();
  double trace = 0.0;
  for (int w = 0; w < nwave; ++w) trace += red[w];
  if (tid == 0 && a.log_scale) {
    a.log_scale[0] = trace > 0.0 ? -0.5 * log(trace) : 0.0;
    a.scale[0] = trace > 0.0 ? 1.0 / sqrt(trace) : 1.0;
  }
  if (tid == 0 && !isfinite(trace)) raise_status(a.status, CBC_ENOTPD);
  const double shift = a.shift_rel * trace;
  __syncthreads();
  double mx = 0.0;
  for (int i = tid; i < k; i += blockDim.x) {
    double2 g = M[i * ld + i];
    g.x += shift;
    g.y = 0.0;
    M[i * ld + i] = g;
    mx = fmax(mx, g.x);
  }
  mx = wmax(mx);
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int w = 0; w < nwave; ++w) m = fmax(m, red[w]);
    sh_thresh = a.drop_rel * m;
  }
  }
  __syncthreads();
  const double thresh = sh_thresh;
  constexpr int RGc = 8;
  const int grp = tid / RGc, gl = tid % RGc, ngrp = blockDim.x / RGc;

  // ---- blocked factorisation ----
  for (int p = 0; p < k; p += NBc) {
    const int pe = min(p + NBc, k);
    if (wave == 0) {
      if (k - p > 64) chol_panel<true>(M, ld, k, p, pe, thresh, dropped, lane);
      else chol_panel<false>(M, ld, k, p, pe, thresh, dropped, lane);
    }
    __syncthreads();
    // trailing update: M[i][l] -= sum_{jj in panel} C[i][jj] conj(C[l][jj]), pe <= l <= i; the
    // panel entries of row i are read once per row
    for (int i = pe + grp; i < k; i += ngrp) {
      double2 ci[NBc];
#pragma unroll
      for (int q = 0; q < NBc; ++q) ci[q] = M[i * ld + min(p + q, pe - 1)];
      for (int l = pe + gl; l <= i; l += RGc) {
        double2 g = M[i * ld + l];
        double2 cl[NBc];
#pragma unroll
        for (int q = 0; q < NBc; ++q) cl[q] = M[l * ld + min(p + q, pe - 1)];
#pragma unroll
        for (int q = 0; q < NBc; ++q) {
          if (p + q < pe) {
            g.x = fma(-ci[q].x, cl[q].x, g.x);
            g.x = fma(-ci[q].y, cl[q].y, g.x);
            g.y = fma(-ci[q].y, cl[q].x, g.y);
            g.y = fma(ci[q].x, cl[q].y, g.y);
          }
        }
        M[i * ld + l] = g;
      }
    }
    __syncthreads();
  }
  if (a.tstamp && tid == 0) a.tstamp[1] = wall_clock64();

  // ---- blocked inverse ----
  // X[r][c] (r > c) lives at M[c][r]; X[r][r] in xd.
  auto xget = [&](int r, int c) -> double2 {
    return r == c ? make_double2(xd[r], 0.0) : M[c * ld + r];
  };
  const int nblk = (k + NBc - 1) / NBc;
  // diagonal blocks: one lane per column of a block (the columns of a triangular inverse are
  // independent); the column is formed in registers by forward substitution
  for (int t = tid; t < nblk * NBc; t += blockDim.x) {
    const int b0 = (t / NBc) * NBc, cl = t % NBc, c = b0 + cl;
    if (c >= k) continue;
    const int b1 = min(b0 + NBc, k);
    if (dropped[c]) {
      xd[c] = 0.0;
      for (int r = c + 1; r < b1; ++r) M[c * ld + r] = make_double2(0.0, 0.0);
      continue;
    }
    const double dc = 1.0 / M[c * ld + c].x;
    xd[c] = dc;
    double2 xr[NBc];   // X[b0 + rr][c]; zero above the diagonal
#pragma unroll
    for (int rr = 0; rr < NBc; ++rr) xr[rr] = rr == cl ? make_double2(dc, 0.0) : make_double2(0.0, 0.0);
#pragma unroll
    for (int rr = 1; rr < NBc; ++rr) {
      const int r = b0 + rr;
      if (rr <= cl || r >= b1) continue;
      if (dropped[r]) {
        M[c * ld + r] = make_double2(0.0, 0.0);
        continue;
      }
      double2 crow[NBc - 1];
#pragma unroll
      for (int ll = 0; ll < rr; ++ll) crow[ll] = M[r * ld + b0 + ll];
      const double ninv = -1.0 / M[r * ld + r].x;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int ll = 0; ll < rr; ++ll) {
        sr += crow[ll].x * xr[ll].x - crow[ll].y * xr[ll].y;
        si += crow[ll].x * xr[ll].y + crow[ll].y * xr[ll].x;
      }
      xr[rr] = make_double2(sr * ninv, si * ninv);
      M[c * ld + r] = xr[rr];
    }
  }
  __syncthreads();
  for (int bi = 1; bi < nblk; ++bi) {
    const int i0 = bi * NBc, i1 = min(i0 + NBc, k), ni = i1 - i0;
    // T[r][c] = sum_{l = col block start}^{i0-1} C[i0+r][l] X[l][c], for c < i0
    for (int idx = tid; idx < ni * i0; idx += blockDim.x) {
      const int r = idx / i0, c = idx % i0;
      const int lstart = (c / NBc) * NBc;
      const double2 xcc = make_double2(xd[c], 0.0);
      double sr = 0.0, si = 0.0;
      for (int lb = max(lstart, c); lb < i0; lb += NBc) {
        double2 cl[NBc], x[NBc];
#pragma unroll
        for (int q = 0; q < NBc; ++q) {
          const int l = min(lb + q, i0 - 1);
          cl[q] = M[(i0 + r) * ld + l];
          x[q] = l == c ? xcc : M[c * ld + l];
        }
#pragma unroll
        for (int q = 0; q < NBc; ++q) {
          if (lb + q < i0) {
            sr = fma(cl[q].x, x[q].x, sr);
            sr = fma(-cl[q].y, x[q].y, sr);
            si = fma(cl[q].x, x[q].y, si);
            si = fma(cl[q].y, x[q].x, si);
          }
        }
      }
      T[r * i0 + c] = make_double2(sr, si);
    }
    __syncthreads();
    // X[i0+r][c] = -sum_{q<=r} X[i0+r][i0+q] T[q][c]
    for (int idx = tid; idx < ni * i0; idx += blockDim.x) {
      const int r = idx / i0, c = idx % i0;
      double sr = 0.0, si = 0.0;
      double2 x[NBc], t[NBc];
#pragma unroll
      for (int q = 0; q < NBc; ++q) {
        const int qq = min(q, r);
        x[q] = xget(i0 + r, i0 + qq);
        t[q] = T[qq * i0 + c];
      }
#pragma unroll
      for (int q = 0; q < NBc; ++q) {
        if (q <= r) {
          sr += x[q].x * t[q].x - x[q].y * t[q].y;
          si += x[q].x * t[q].y + x[q].y * t[q].x;
        }
      }
      M[c * ld + i0 + r] = make_double2(-sr, -si);
    }
    __syncthreads();
  }
  if (a.tstamp && tid == 0) a.tstamp[2] = wall_clock64();
  for (int idx = tid; idx < k * k; idx += blockDim.x) {
    const int i = idx / k, c = idx % k;
    double2 v = make_double2(0.0, 0.0);
    if (i == c) v = make_double2(xd[c], 0.0);
    else if (i > c) v = M[c * ld + i];
    a.Cinv[(size_t)i * gld + c] = v;
  }
  if (a.ndrop && tid == 0) {
    int nd = 0;
    for (int j = 0; j < k; ++j) nd += dropped[j];
    a.ndrop[0] += nd;
  }
  __syncthreads();
  if (a.tstamp && tid == 0) a.tstamp[3] = wall_clock64();
}

// ---- blocked factorisation for k > CHOL_LDS_MAX ------------------------------------------------
// Right-looking, by blocks of CHOL_NB columns: the diagonal block is factorised and inverted by the
// LDS kernel, the panel below it is C_ip = G_ip C_pp^{-H} and the trailing matrix is updated with
// G -= C_ip C_jp^H (both on the contraction GEMM in dense mode, FP64). Block row i of the inverse is
// then X_i,<i = -X_ii (C_i,<i X_<i,<i). Pivots are dropped against the same absolute threshold as
// the unblocked algorithm (drop_rel times the largest shifted diagonal entry), so this is the same
// computation in another order.
static constexpr int CHOL_NB = 64;

size_t chol_work_doubles(int k) {
  return 2 * (size_t)k * k + 2 * (size_t)CHOL_NB * k + 16;
}

// trace -> log-scale / scale, diagonal shift, pivot threshold (one workgroup per instance)
// A re-orthogonalisation pass (no shift) of the blocked factorisation whose Gram is the identity to
// rounding (the criterion of the LDS kernel): C^{-1} = I is written and `flag` set, so that the
// blocked steps after it do nothing; otherwise `flag` is cleared. One workgroup per instance.
__global__ __launch_bounds__(CHOL_THREADS) void k_chol_ident(CholArgs a0, int* flag) {
  const CholArgs a = chol_inst(a0, blockIdx.x);
  flag = inst_ptr(flag, a0.bs, blockIdx.x);
  __shared__ double red[32];
  const int k = a.k, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  double dev = 0.0;
  for (int i = tid; i < k * k; i += blockDim.x) {
    const int r = i / k, c = i % k;
    const double2 g = a.G[(size_t)r * k + c];
    dev = fmax(dev, fmax(fabs(g.x - (r == c ? 1.0 : 0.0)), fabs(g.y)));
  }
  dev = wmax(dev);
  if (lane == 0) red[wave] = dev;
  __syncthreads();
  double m = 0.0;
  for (int w = 0; w < nwave; ++w) m = fmax(m, red[w]);
  const bool ident = m <= 4.0 * k * DBL_EPSILON * 0.5;   // NaN entries fail the test
  if (ident)
    for (int idx = tid; idx < k * k; idx += blockDim.x)
      a.Cinv[idx] = make_double2(idx / k == idx % k ? 1.0 : 0.0, 0.0);
  if (tid == 0) *flag = ident ? 1 : 0;
}

__global__ __launch_bounds__(CHOL_THREADS) void k_chol_prep(CholArgs a0, double* thresh_out) {
  const CholArgs a = chol_inst(a0, blockIdx.x);
  if (a.skip && *a.skip) return;
  thresh_out = inst_ptr(thresh_out, a0.bs, blockIdx.x);
  __shared__ double red[32];
  __shared__ double sh_trace;
  const int k = a.k, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  double tr = 0.0;
  for (int i = tid; i < k; i += blockDim.x) tr += a.G[(size_t)i * k + i].x;
  tr = wsum(tr);
  if (lane == 0) red[wave] = tr;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < nwave; ++w) t += red[w];
    sh_trace = t;
    if (!isfinite(t)) raise_status(a.status, CBC_ENOTPD);
    if (a.log_scale) {
      a.log_scale[0] = t > 0.0 ? -0.5 * log(t) : 0.0;
      a.scale[0] = t > 0.0 ? 1.0 / sqrt(t) : 1.0;
    }
  }
  __syncthreads();
  const double shift = a.shift_rel * sh_trace;
  double mx = 0.0;
  for (int i = tid; i < k; i += blockDim.x) {
    double2 g = a.G[(size_t)i * k + i];
    g.x += shift;
    g.y = 0.0;
    a.G[(size_t)i * k + i] = g;
    mx = fmax(mx, g.x);
  }
  mx = wmax(mx);
  __syncthreads();
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int w = 0; w < nwave; ++w) m = fmax(m, red[w]);
    thresh_out[0] = a.drop_rel * m;
  }
}

static size_t chol_lds_bytes(int k) {
  return (size_t)k * (k + 1) * sizeof(double2) + (size_t)k * sizeof(double) +
         (size_t)((k + 3) & ~3) * sizeof(int) + (size_t)k * NBc * sizeof(double2);
}

// dense FP64 GEMM on sub-blocks (row-major strides), same batch layout as the factorisation
static hipError_t dense_gemm(const CholArgs& a, int M, int N, int K, const double2* A, int64_t sAm,
                             int64_t sAk, const double2* B, int64_t sBk, int64_t sBn, int conjB,
                             double2* C, int64_t sCm, int64_t sCn, double alpha, int accum,
                             hipStream_t st) {
  GemmArgs g;
  g.A = A; g.B = B; g.C = C; g.M = M; g.N = N; g.K = K;
  g.offAm = g.offAk = g.offBk = g.offBn = g.offCm = g.offCn = nullptr;
  g.sAm = sAm; g.sAk = sAk; g.sBk = sBk; g.sBn = sBn; g.sCm = sCm; g.sCn = sCn;
  g.conjA = 0; g.conjB = conjB;
  g.a_kfast = sAk == 1;
  g.b_kfast = sBk == 1;
  g.alpha_dev = nullptr; g.alpha_dev2 = nullptr; g.alpha = alpha;
  g.batch = a.batch;
  g.bsA = g.bsB = g.bsC = a.bs;
  g.bsAlpha = g.bsAlpha2 = 0;
  g.accum = accum;
  g.skip = a.skip;
  g.bsSkip = a.bs;
  return launch_gemm(g, DT_C128, DT_C128, DT_C128, DT_C128, GEMM_TILE32, st);
}

hipError_t launch_chol_inv(const CholArgs& a, hipStream_t st) {
  if (a.k <= 0 || a.batch <= 0) return hipSuccess;
  if (a.k <= CHOL_LDS_MAX) {
    const size_t lds = chol_lds_bytes(a.k);
    (void)hipFuncSetAttribute((const void*)k_chol_inv_lds,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_chol_inv_lds, dim3(a.batch), dim3(CHOL_THREADS), lds, st, a);
    return hipGetLastError();
  }
  if (!a.work) return hipErrorInvalidValue;
  const int k = a.k;
  double2* G = a.G;
  double2* X = a.Cinv;
  double2* Cf = a.work;                                      // k x k factor panels
  double2* T = a.work + (size_t)k * k;                       // CHOL_NB x k
  double* thr = reinterpret_cast<double*>(T + (size_t)CHOL_NB * k);
  int* flag = reinterpret_cast<int*>(thr + 1);
  hipError_t e = launch_zero(X, (int64_t)16 * k * k, a.batch, a.bs, st);
  if (e != hipSuccess) return e;
  CholArgs b = a;
  if (a.shift_rel == 0.0 && !a.thresh_dev) {
    // a re-orthogonalisation pass: the identity shortcut, and every later step skips where it holds
    hipLaunchKernelGGL(k_chol_ident, dim3(a.batch), dim3(CHOL_THREADS), 0, st, a, flag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    b.skip = flag;
  }
  hipLaunchKernelGGL(k_chol_prep, dim3(b.batch), dim3(CHOL_THREADS), 0, st, b, thr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = chol_lds_bytes(CHOL_NB);
  (void)hipFuncSetAttribute((const void*)k_chol_inv_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  for (int o = 0; o < k; o += CHOL_NB) {
    const int bp = k - o < CHOL_NB ? k - o : CHOL_NB;
    CholArgs d = b;
    d.G = G + (size_t)o * k + o;
    d.Cinv = X + (size_t)o * k + o;
    d.k = bp;
    d.ld = k;
    d.thresh_dev = thr;
    d.log_scale = nullptr;
    d.scale = nullptr;
    d.work = nullptr;
    d.tstamp = nullptr;
    hipLaunchKernelGGL(k_chol_inv_lds, dim3(a.batch), dim3(CHOL_THREADS), lds, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int r0 = o + bp, rows = k - r0;
    if (rows <= 0) break;
    // panel: Cf[r, c] = sum_l G[r, l] conj(X_pp[c, l])
    e = dense_gemm(b, rows, bp, bp, G + (size_t)r0 * k + o, k, 1, X + (size_t)o * k + o, 1, k, 1,
                   Cf + (size_t)r0 * k + o, k, 1, 1.0, 0, st);
    if (e != hipSuccess) return e;
    // trailing: G[r, r'] -= sum_c Cf[r, c] conj(Cf[r', c])
    e = dense_gemm(b, rows, rows, bp, Cf + (size_t)r0 * k + o, k, 1, Cf + (size_t)r0 * k + o, 1, k, 1,
                   G + (size_t)r0 * k + r0, k, 1, -1.0, 1, st);
    if (e != hipSuccess) return e;
  }
  // inverse, block rows i >= 1: T = Cf[i, <i] X[<i, <i]; X[i, <i] = -X_ii T
  for (int oi = CHOL_NB; oi < k; oi += CHOL_NB) {
    const int bi = k - oi < CHOL_NB ? k - oi : CHOL_NB;
    e = dense_gemm(b, bi, oi, oi, Cf + (size_t)oi * k, k, 1, X, k, 1, 0, T, k, 1, 1.0, 0, st);
    if (e != hipSuccess) return e;
    e = dense_gemm(b, bi, oi, bi, X + (size_t)oi * k + oi, k, 1, T, k, 1, 0, X + (size_t)oi * k, k, 1,
                   -1.0, 0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------------------------------------
// elementwise helpers

__global__ void k_convert(const void* src, int ts, void* dst, int td, int64_t n, int64_t ss,
                          int64_t ds) {
  const int b = blockIdx.y;
  src = inst_ptr(src, ss, b);
  dst = inst_ptr(dst, ds, b);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 v;
  if (ts == DT_C128) v = reinterpret_cast<const double2*>(src)[i];
  else {
    const float2 f = reinterpret_cast<const float2*>(src)[i];
    v = make_double2(f.x, f.y);
  }
  if (td == DT_C128) reinterpret_cast<double2*>(dst)[i] = v;
  else reinterpret_cast<float2*>(dst)[i] = make_float2((float)v.x, (float)v.y);
}

hipError_t launch_convert(const void* src, DType ts, void* dst, DType td, int64_t n, int batch,
                          int64_t ss, int64_t ds, hipStream_t st) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)((n + 255) / 256), batch), dim3(256), 0, st, src,
                     (int)ts, dst, (int)td, n, ss, ds);
  return hipGetLastError();
}

// x *= 1 / ||x||_F in place. The sum of squares is taken in FP64 in a fixed order: block b of the
// first kernel sums the elements b, b + nb*256, ... (nb = norm_blocks(n)) into part[b]; every block
// of the second adds part[0..nb) in order, so all blocks compute the same factor, and scales its
// share of x. The factor goes to scale[0] and its logarithm to logs[0] where those are given. A zero
// norm leaves x as it is (factor 1); a non-finite one also stores CBC_ENOTPD in the status word.
static constexpr int NORM_THREADS = 256;

__global__ __launch_bounds__(NORM_THREADS) void k_norm_partial(const void* x, int t, int64_t n,
                                                               double* part) {
  __shared__ double red[NORM_THREADS / 64];
  const int tid = threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * NORM_THREADS;
  double s = 0.0;
  if (t == DT_C128) {
    const double2* p = reinterpret_cast<const double2*>(x);
    for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + tid; i < n; i += stride)
      s += p[i].x * p[i].x + p[i].y * p[i].y;
  } else {
    const float2* p = reinterpret_cast<const float2*>(x);
    for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + tid; i < n; i += stride) {
      const double a = p[i].x, b = p[i].y;
      s += a * a + b * b;
    }
  }
  s = wsum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < NORM_THREADS / 64; ++w) tot += red[w];
    part[blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(NORM_THREADS) void k_norm_apply(void* x, int t, int64_t n,
                                                             const double* part, int nb,
                                                             double* scale, double* logs,
                                                             int* status) {
  __shared__ double fac;
  const int tid = threadIdx.x;
  if (tid == 0) {
    double tot = 0.0;
    for (int b = 0; b < nb; ++b) tot += part[b];
    double f = 1.0;
    if (isfinite(tot) && tot > 0.0) f = 1.0 / sqrt(tot);
    fac = f;
    if (blockIdx.x == 0) {
      if (!isfinite(tot)) raise_status(status, CBC_ENOTPD);
      if (scale) scale[0] = f;
      if (logs) logs[0] = log(f);
    }
  }
  __syncthreads();
  const double f = fac;
  const int64_t stride = (int64_t)gridDim.x * NORM_THREADS;
  if (t == DT_C128) {
    double2* p = reinterpret_cast<double2*>(x);
    for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + tid; i < n; i += stride)
      p[i] = make_double2(p[i].x * f, p[i].y * f);
  } else {
    float2* p = reinterpret_cast<float2*>(x);
    const float g = (float)f;
    for (int64_t i = (int64_t)blockIdx.x * NORM_THREADS + tid; i < n; i += stride)
      p[i] = make_float2(p[i].x * g, p[i].y * g);
  }
}

int norm_blocks(int64_t n) {
  const int64_t b = (n + NORM_THREADS - 1) / NORM_THREADS;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, NORM_MAX_BLOCKS));
}

hipError_t launch_normalize(void* x, DType t, int64_t n, double* part, double* scale, double* logs,
                            int* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int nb = norm_blocks(n);
  hipLaunchKernelGGL(k_norm_partial, dim3(nb), dim3(NORM_THREADS), 0, st, x, (int)t, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_norm_apply, dim3(nb), dim3(NORM_THREADS), 0, st, x, (int)t, n, part, nb,
                     scale, logs, status);
  return hipGetLastError();
}

__global__ void k_fill_identity(void* dst, int t, int rows, int cols, int64_t ds) {
  dst = inst_ptr(dst, ds, blockIdx.y);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  const double v = (r == c) ? 1.0 : 0.0;
  if (t == DT_C128) reinterpret_cast<double2*>(dst)[i] = make_double2(v, 0.0);
  else reinterpret_cast<float2*>(dst)[i] = make_float2((float)v, 0.0f);
}

hipError_t launch_fill_identity(void* dst, DType t, int rows, int cols, int batch, int64_t ds,
                                hipStream_t st) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0 || batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_identity, dim3((unsigned)((n + 255) / 256), batch), dim3(256), 0, st,
                     dst, (int)t, rows, cols, ds);
  return hipGetLastError();
}

__global__ void k_zero_words(uint32_t* p, int64_t n, int64_t ds) {
  p = inst_ptr(p, ds, blockIdx.y);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_zero(void* dst, int64_t bytes, int batch, int64_t ds, hipStream_t st) {
  const int64_t nw = (bytes + 3) / 4;
  if (nw <= 0 || batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((nw + 255) / 256), batch), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(dst), nw, ds);
  return hipGetLastError();
}

// dst[(b, a, r)] = src[(a, b, r)] * exp(-sum logs)
__global__ void k_report_header(char* ws, uint32_t magic, int n_rec, int64_t rec_off,
                                int64_t rec_bytes, int64_t ds) {
  ws += ds * (int64_t)blockIdx.y;
  uint32_t* rec = reinterpret_cast<uint32_t*>(ws + rec_off);
  const int64_t nw = (int64_t)n_rec * rec_bytes / 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (int64_t)gridDim.x * blockDim.x)
    rec[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < 16) {
    uint32_t* h = reinterpret_cast<uint32_t*>(ws);
    uint32_t v = 0u;
    if (threadIdx.x == 0) v = magic;
    else if (threadIdx.x == 3) v = (uint32_t)n_rec;
    else if (threadIdx.x == 4) v = (uint32_t)(uint64_t)rec_off;
    else if (threadIdx.x == 5) v = (uint32_t)((uint64_t)rec_off >> 32);
    h[threadIdx.x] = v;
  }
}

hipError_t launch_report_header(void* ws, uint32_t magic, int n_rec, int64_t rec_off,
                                int64_t rec_bytes, int batch, int64_t ds, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const int64_t nw = (int64_t)n_rec * rec_bytes / 4;
  const int blocks = (int)std::min<int64_t>(64, std::max<int64_t>(1, (nw + 255) / 256));
  hipLaunchKernelGGL(k_report_header, dim3(blocks, batch), dim3(256), 0, st, (char*)ws, magic,
                     n_rec, rec_off, rec_bytes, ds);
  return hipGetLastError();
}

__global__ void k_write_out(const void* src, int ts, int a, int b, int64_t rest, double2* dst,
                            const double* logs, int nlogs, int64_t ss, int64_t ds, int64_t ls) {
  const int inst = blockIdx.y;
  src = inst_ptr(src, ss, inst);
  dst = inst_ptr(dst, ds, inst);
  logs = inst_ptr(logs, ls, inst);
  __shared__ double sh_f;
  if (threadIdx.x == 0) {
    double l = 0.0;
    if (logs)
      for (int i = 0; i < nlogs; ++i) l += logs[i];
    sh_f = exp(-l);
  }
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)a * b * rest;
  if (idx >= n) return;
  const int64_t r = idx % rest;
  const int64_t ab = idx / rest;
  const int64_t ib = ab / a, ia = ab % a;     // dst index (ib, ia, r)
  const int64_t sidx = (ia * b + ib) * rest + r;
  double2 v;
  if (ts == DT_C128) v = reinterpret_cast<const double2*>(src)[sidx];
  else {
    const float2 f = reinterpret_cast<const float2*>(src)[sidx];
    v = make_double2(f.x, f.y);
  }
  const double f = sh_f;
  dst[idx] = make_double2(v.x * f, v.y * f);
}

hipError_t launch_write_out(const void* src, DType ts, int a, int b, int64_t rest, double2* dst,
                            const double* logs, int nlogs, int batch, int64_t ss, int64_t ds,
                            int64_t ls, hipStream_t st) {
  const int64_t n = (int64_t)a * b * rest;
  if (n <= 0 || batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_write_out, dim3((unsigned)((n + 255) / 256), batch), dim3(256), 0, st, src,
                     (int)ts, a, b, rest, dst, logs, nlogs, ss, ds, ls);
  return hipGetLastError();
}

}  // namespace cbc
