// Two-stage reduction of an FP64 Hermitian Gram matrix to real symmetric tridiagonal form (for
// Grams larger than the single-workgroup reduction's LDS limit), and the back-transformation of the
// eigenvectors through both stages.
//
// The truncation of Sec. III A keeps the top-k eigenspace of the Gram of the joined-leg matrix. Any
// unitary similarity G = Q T Q^H with T real tridiagonal gives it: T's eigenvectors y map to G's as
// u = Q y. Here Q = Q1 Q2:
//   stage 1, dense -> band of half-bandwidth NB: the block below the band of column panel p (rows
//     r0 = (p+1) NB .. s-1, columns p NB .. p NB + NB - 1) is factored by Householder QR,
//     Q_p = I - V T V^H (compact WY form, T upper triangular), and the trailing matrix is updated
//     two-sidedly, A22 <- Q_p^H A22 Q_p = A22 - V W^H - W V^H with X = A22 V T and
//     W = X - V (T^H V^H X) / 2. Four launches per panel: the panel QR (one workgroup, rows in
//     registers, one workgroup-wide reduction per column), X (row blocks over the GPU, forming V T
//     on the way, with partial sums of V^H X), W, and the rank-2NB update as one FP64 MFMA product
//     on the contraction kernel.
//   stage 2, band -> tridiagonal by bulge chasing: sweep i annihilates column i below the first
//     sub-diagonal with a reflector on rows i+1 .. i+NB, and chases the resulting bulge down the band
//     in steps of NB rows (each step: the previous reflector applied from the right to the block
//     below it, a new reflector from that block's first column applied from the left, and the
//     two-sided update of the diagonal block). Step t of sweep i touches only rows that step t+1 of
//     sweep i-1 has finished with, so one workgroup runs 16 sweeps at once, one per wave, each wave
//     waiting on its predecessor's step counter in LDS; the band stays in L2.
// Every reflector follows LAPACK's convention H = I - tau v v^H, H^H x = beta e_1, beta real, so the
// tridiagonal comes out real.
#include "eig_common.h"

namespace cbc {

static constexpr int NB = 16;        // half-bandwidth of the intermediate band matrix
static constexpr int LDB = 2 * NB;   // stored sub-diagonals of the band (bulges reach 2 NB - 1)
static constexpr int XR = 16;        // rows of X per workgroup (one per wave)
// eigenvectors per back-transformation workgroup: one (k workgroups over the GPU; measured on
// MI355X at s = 1024, k = 256: eigenvectors and back-transformation 4.8 ms with four, 3.0 with two,
// 2.0 with one)
static constexpr int BT_NV = 1;

__host__ __device__ inline int band_T2(int s) { return (s - 1 + NB - 1) / NB; }
// panels whose block below the band has at least two rows
__host__ __device__ inline int band_npan(int s) { return s >= NB + 2 ? (s - 2) / NB : 0; }
__host__ __device__ inline int band_nxblk(int s) { return (s + XR - 1) / XR; }

// Scratch of the two-stage path, after the common eigensolver layout.
struct BandWork {
  double2* V2;    // stage-2 reflectors, (s-1) sweeps x T2 steps x NB (zero past the block's end)
  double2* tau2;  // (s-1) x T2
  double2* band;  // s x LDB, column-major lower band: A[c + d, c] at band[c * LDB + d]
  double2* T1;    // stage-1 triangular factors, npan x NB x NB
  double2* Z;     // s x 3NB: [V | W | V] of the current panel (rows relative to r0)
  double2* VT;    // s x NB: V T
  double2* X;     // s x NB: A22 V T
  double2* Sp;    // nxblk x NB x NB: per-workgroup partial sums of V^H X
};
__host__ __device__ inline size_t band_align(size_t d) { return (d + 15) & ~(size_t)15; }
__host__ __device__ inline BandWork band_layout(double* w, int s) {
  BandWork B;
  const size_t T2 = band_T2(s), np = band_npan(s) > 0 ? band_npan(s) : 1;
  double* q = w;
  auto take = [&](size_t cplx) {
    double2* r = reinterpret_cast<double2*>(q);
    q += band_align(2 * cplx);
    return r;
  };
  B.V2 = take((size_t)(s - 1) * T2 * NB);
  B.tau2 = take((size_t)(s - 1) * T2);
  B.band = take((size_t)s * LDB);
  B.T1 = take(np * NB * NB);
  B.Z = take((size_t)s * 3 * NB);
  B.VT = take((size_t)s * NB);
  B.X = take((size_t)s * NB);
  B.Sp = take((size_t)band_nxblk(s) * NB * NB);
  return B;
}
size_t band_work_doubles(int s) {
  double* base = nullptr;
  const BandWork B = band_layout(base + 0, s);
  return (size_t)(reinterpret_cast<double*>(B.Sp) - base) +
         band_align(2 * (size_t)band_nxblk(s) * NB * NB) + 16;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// conj(a) * b
__device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc - a * b
__device__ __forceinline__ double2 cfms(double2 a, double2 b, double2 acc) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 cscale(double2 a, double f) { return make_double2(a.x * f, a.y * f); }
__device__ __forceinline__ double2 shfl_z(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}
__device__ __forceinline__ double2 shfl_xor_z(double2 v, int m) {
  return make_double2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}
__device__ __forceinline__ double2 sum16_z(double2 v) { return make_double2(sum16(v.x), sum16(v.y)); }

// Sixteen doubles summed over the wave by recursive halving: afterwards every lane l holds the wave
// total of value (l >> 2) & 15 in v[0].
template <int O, int M>
__device__ __forceinline__ void halve_stage(double* v, int lane) {
  const bool hi = (lane & O) != 0;
#pragma unroll
  for (int i = 0; i < M / 2; ++i) {
    const double send = hi ? v[i] : v[i + M / 2];
    const double keep = hi ? v[i + M / 2] : v[i];
    v[i] = keep + __shfl_xor(send, O, 64);
  }
}
// Eight doubles: afterwards every lane l holds the wave total of value (l >> 3) & 7 in v[0].
__device__ __forceinline__ void wave_sum8x(double v[8], int lane) {
  halve_stage<32, 8>(v, lane);
  halve_stage<16, 4>(v, lane);
  halve_stage<8, 2>(v, lane);
  v[0] += __shfl_xor(v[0], 4, 64);
  v[0] += __shfl_xor(v[0], 2, 64);
  v[0] += __shfl_xor(v[0], 1, 64);
}
__device__ __forceinline__ void wave_sum16x(double v[16], int lane) {
  halve_stage<32, 16>(v, lane);
  halve_stage<16, 8>(v, lane);
  halve_stage<8, 4>(v, lane);
  halve_stage<4, 2>(v, lane);
  v[0] += __shfl_xor(v[0], 2, 64);
  v[0] += __shfl_xor(v[0], 1, 64);
}

// Householder scalars for x (alpha = x_0, xn2 = |x_1..|^2): tau, beta and 1/(alpha - beta); the
// identity (tau = 0) when x_1.. vanish and alpha is real.
__device__ __forceinline__ void reflector_scalars(double2 alpha, double xn2, double2& tau, double& beta,
                                                  double2& scal) {
  tau = make_double2(0.0, 0.0);
  scal = make_double2(0.0, 0.0);
  beta = alpha.x;
  if (xn2 == 0.0 && alpha.y == 0.0) return;
  const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
  beta = alpha.x >= 0.0 ? -nrm : nrm;
  tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
  const double ar = alpha.x - beta, ai = alpha.y;
  const double den = ar * ar + ai * ai;
  scal = make_double2(ar / den, -ai / den);
}

// a wave-uniform double moved to scalar registers (keeps per-column constants out of the vector
// register file, which holds the panel rows)
__device__ __forceinline__ double uni(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ __forceinline__ double2 uni2(double2 v) { return make_double2(uni(v.x), uni(v.y)); }

// ---- stage 1: panel QR --------------------------------------------------------------------------
// Thread t holds rows t + TH q (q < R) of the panel (NB complex each) in registers. Column C:
// one reduction over the rows below the pivot gives |x_1..|^2, x^H a_j for the later columns j and
// V_q^H x for the earlier reflectors q (needed for T); the pivot row comes from its owner through
// LDS. Columns are template parameters so that every register index is static.
template <int R>
struct PanelState {
  double2 P[R][NB];
};

template <int R, int TH, int C>
__device__ __forceinline__ void panel_column(PanelState<R>& S, int h, int tid, int lane, int wave,
                                             double (*red)[32], double* tot, double2 (*piv)[NB],
                                             double2 (*Tm)[NB], double2 (*Gq)[NB]) {
  double2* pv = piv[C & 1];
  if (tid == C) {
#pragma unroll
    for (int j = 0; j < NB; ++j) pv[j] = S.P[0][j];
  }
  // value k (0..14): V_k^H x for k < C (reflector k is stored in column k), x^H a_{k+1} otherwise;
  // value 15: |x|^2. Each is summed over the thread's rows, then over 16-lane rows by DPP; lane 0
  // of every row stores its partial.
  const bool row0 = (lane & 15) == 0;
  double* rp = red[wave * 4 + (lane >> 4)];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = tid + TH * q;
      if (r > C && r < h) {
        const double2 x = S.P[q][C];
        if (k == 15) {
          re += x.x * x.x + x.y * x.y;
        } else {
          const double2 pr = k < C ? cjmul(S.P[q][k < C ? k : 0], x)
                                   : cjmul(x, S.P[q][k + 1 < NB ? k + 1 : 0]);
          re += pr.x;
          im += pr.y;
        }
      }
    }
    re = sum16(re);
    if (row0) rp[2 * k] = re;
    if (k < 15) {
      im = sum16(im);
      if (row0) rp[2 * k + 1] = im;
    }
  }
  __syncthreads();
  if (tid < 32 && tid != 31) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < 4 * (TH / 64); ++w) acc += red[w][tid];
    tot[tid] = acc;
  }
  __syncthreads();
  const double2 alpha = uni2(pv[C]);
  double2 tau, scal;
  double beta;
  reflector_scalars(alpha, tot[30], tau, beta, scal);
  const double2 ctau = make_double2(tau.x, -tau.y);
  // reflector entries of the own rows (the pivot row's is 1)
  double2 vr[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + TH * q;
    vr[q] = make_double2(0.0, 0.0);
    if (r == C) {
      vr[q] = make_double2(1.0, 0.0);
      S.P[q][C] = make_double2(beta, 0.0);
    } else if (r > C && r < h) {
      vr[q] = cmul(S.P[q][C], scal);
      S.P[q][C] = vr[q];
    }
  }
  // a_j -= conj(tau) v (v^H a_j), v^H a_j = a_Cj + conj(scal) x^H a_j
#pragma unroll
  for (int j = C + 1; j < NB; ++j) {
    const double2 dj = make_double2(tot[2 * (j - 1)], tot[2 * (j - 1) + 1]);
    const double2 zj = cadd(pv[j], cjmul(scal, dj));
    const double2 f = uni2(cmul(ctau, zj));
#pragma unroll
    for (int q = 0; q < R; ++q) S.P[q][j] = cfms(vr[q], f, S.P[q][j]);
  }
  // for T (formed after the last column): tau_C and V_q^H v_C = conj(V_q[C]) + scal V_q^H x, q < C
  if (tid == 0) Tm[C][C] = tau;
  if (tid < C)
    Gq[C][tid] = cadd(make_double2(pv[tid].x, -pv[tid].y),
                      cmul(scal, make_double2(tot[2 * tid], tot[2 * tid + 1])));
}

template <int R, int TH, int C>
__device__ __forceinline__ void panel_columns(PanelState<R>& S, int ncol, int h, int tid, int lane,
                                              int wave, double (*red)[32], double* tot,
                                              double2 (*piv)[NB], double2 (*Tm)[NB],
                                              double2 (*Gq)[NB]) {
  if constexpr (C < NB) {
    if (C < ncol) {
      panel_column<R, TH, C>(S, h, tid, lane, wave, red, tot, piv, Tm, Gq);
      panel_columns<R, TH, C + 1>(S, ncol, h, tid, lane, wave, red, tot, piv, Tm, Gq);
    }
  }
}

template <int R, int TH>
__global__ __launch_bounds__(TH) void k_band_panel(EigArgs a0, int p) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int s = a.s;
  const int c0 = p * NB, r0 = c0 + NB, h = s - r0, ncol = min(NB, h);
  const BandWork B = band_layout(a.work + eig_base_doubles(s, a.kmax), s);
  double2* __restrict__ G = a.G;
  __shared__ double red[4 * (TH / 64)][32];
  __shared__ double tot[32];
  __shared__ double2 piv[2][NB];
  __shared__ double2 Tm[NB][NB];
  __shared__ double2 Gq[NB][NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  long long ts0 = a.tstamp && tid == 0 ? wall_clock64() : 0, ts1 = 0;
  // accumulated phase durations (time stamps of thread 0, optional)
  auto phase = [&](int slot) {
    if (a.tstamp && tid == 0) {
      ts1 = wall_clock64();
      atomicAdd(reinterpret_cast<unsigned long long*>(a.tstamp + slot), (unsigned long long)(ts1 - ts0));
      ts0 = ts1;
    }
  };
  PanelState<R> S;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + TH * q;
#pragma unroll
    for (int j = 0; j < NB; ++j)
      S.P[q][j] = r < h ? G[(size_t)(r0 + r) * s + c0 + j] : make_double2(0.0, 0.0);
  }
  if (tid < NB * NB) Tm[tid / NB][tid % NB] = make_double2(0.0, 0.0);
  __syncthreads();
  phase(8);
  panel_columns<R, TH, 0>(S, ncol, h, tid, lane, wave, red, tot, piv, Tm, Gq);
  __syncthreads();
  phase(9);
  // T column by column: T[i, C] = -tau_C sum_{i <= k < C} T[i, k] (V_k^H v_C); lane i owns row i
  if (tid < NB) {
    const int i = tid;
    for (int C = 1; C < ncol; ++C) {
      if (i < C) {
        double2 acc = make_double2(0.0, 0.0);
        for (int k = i; k < C; ++k) acc = cfma(Tm[i][k], Gq[C][k], acc);
        const double2 tc = Tm[C][C];
        Tm[i][C] = make_double2(-(tc.x * acc.x - tc.y * acc.y), -(tc.x * acc.y + tc.y * acc.x));
      }
    }
  }
  __syncthreads();
  phase(10);
  // R and the reflectors back into G (LAPACK layout) and [V | 0 | V] into Z
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = tid + TH * q;
    if (r >= h) continue;
    double2* ve = S.P[q];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      G[(size_t)(r0 + r) * s + c0 + j] = ve[j];
      ve[j] = j >= ncol || r < j ? make_double2(0.0, 0.0)
                                 : (r == j ? make_double2(1.0, 0.0) : ve[j]);
    }
    double2* z = B.Z + (size_t)r * 3 * NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      z[j] = ve[j];
      z[NB + j] = make_double2(0.0, 0.0);
      z[2 * NB + j] = ve[j];
    }
  }
  if (tid < NB * NB) B.T1[(size_t)p * NB * NB + tid] = Tm[tid / NB][tid % NB];
  __syncthreads();
  phase(11);
}

// ---- stage 1: X = A22 (V T), one row of X per wave, and partial sums of V^H X per workgroup -------
// V T is formed in chunks of 64 rows from the explicit V and T and staged through LDS (transposed,
// so a wave reads 64 consecutive entries of one column), shared by the workgroup's 16 rows.
__global__ __launch_bounds__(1024) void k_band_x(EigArgs a0, int p) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int s = a.s;
  const int r0 = (p + 1) * NB, h = s - r0;
  const BandWork B = band_layout(a.work + eig_base_doubles(s, a.kmax), s);
  __shared__ double2 xs[XR][NB];
  __shared__ double2 vts[NB][64];
  __shared__ double2 Ts[NB][NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = blockIdx.x * XR + wave;
  if (tid < NB * NB) Ts[tid / NB][tid % NB] = B.T1[(size_t)p * NB * NB + tid];
  __syncthreads();
  double2 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = make_double2(0.0, 0.0);
  const double2* __restrict__ arow = a.G + (size_t)(r0 + min(i, h - 1)) * s + r0;
  for (int k0 = 0; k0 < h; k0 += 64) {
    {
      // (V T)[k0 + kk, j] = sum_{m <= j} V[k0 + kk, m] T[m, j]
      const int kk = tid >> 4, j = tid & 15;
      double2 acc = make_double2(0.0, 0.0);
      if (k0 + kk < h) {
        const double2* __restrict__ vrow = B.Z + (size_t)(k0 + kk) * 3 * NB;
        for (int m = 0; m <= j; ++m) acc = cfma(vrow[m], Ts[m][j], acc);
      }
      vts[j][kk] = acc;
    }
    __syncthreads();
    const double2 x = i < h && k0 + lane < h ? arow[k0 + lane] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = cfma(x, vts[j][lane], acc[j]);
    __syncthreads();
  }
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[2 * k] = acc[half * 8 + k].x;
      v[2 * k + 1] = acc[half * 8 + k].y;
    }
    wave_sum16x(v, lane);
    if ((lane & 3) == 0) reinterpret_cast<double*>(xs[wave])[half * 16 + ((lane >> 2) & 15)] = v[0];
  }
  __syncthreads();
  if (i < h && lane < NB) B.X[(size_t)i * NB + lane] = xs[wave][lane];
  if (tid < NB * NB) {
    const int ra = tid / NB, cb = tid % NB;
    double2 sacc = make_double2(0.0, 0.0);
    for (int w = 0; w < XR; ++w) {
      const int ii = blockIdx.x * XR + w;
      if (ii < h) sacc = cadd(sacc, cjmul(B.Z[(size_t)ii * 3 * NB + ra], xs[w][cb]));
    }
    B.Sp[(size_t)blockIdx.x * NB * NB + tid] = sacc;
  }
}

// ---- stage 1: W = X - V (T^H S) / 2 with S = V^H X summed over the X workgroups in order ----------
// Every workgroup forms S and M = T^H S / 2 itself (the partial sums stay in L2), then 64 rows of W
// with 16 threads per row (one column of W each).
static constexpr int WROWS = 64;
__global__ __launch_bounds__(1024) void k_band_w(EigArgs a0, int p) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int s = a.s;
  const int r0 = (p + 1) * NB, h = s - r0;
  const int nblk = (h + XR - 1) / XR;
  const BandWork B = band_layout(a.work + eig_base_doubles(s, a.kmax), s);
  __shared__ double2 S[NB][NB], M[NB][NB];
  const int tid = threadIdx.x;
  if (tid < NB * NB) {
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < nblk; ++b) acc = cadd(acc, B.Sp[(size_t)b * NB * NB + tid]);
    S[tid / NB][tid % NB] = acc;
  }
  __syncthreads();
  if (tid < NB * NB) {
    const int ra = tid / NB, cb = tid % NB;
    const double2* T = B.T1 + (size_t)p * NB * NB;
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k <= ra; ++k) acc = cadd(acc, cjmul(T[k * NB + ra], S[k][cb]));
    M[ra][cb] = make_double2(0.5 * acc.x, 0.5 * acc.y);
  }
  __syncthreads();
  const int r = blockIdx.x * WROWS + (tid >> 4), cb = tid & 15;
  if (r < h) {
    double2* z = B.Z + (size_t)r * 3 * NB;
    double2 w = B.X[(size_t)r * NB + cb];
#pragma unroll
    for (int k = 0; k < NB; ++k) w = cfms(z[k], M[k][cb], w);
    z[NB + cb] = w;
  }
}

// ---- band extraction: A[c + d, c], d <= NB, into the column-major band (zero above NB) ----------
__global__ void k_band_extract(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int s = a.s;
  const BandWork B = band_layout(a.work + eig_base_doubles(s, a.kmax), s);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)s * LDB) return;
  const int c = (int)(idx / LDB), d = (int)(idx % LDB);
  double2 v = make_double2(0.0, 0.0);
  if (d <= NB && c + d < s) v = a.G[(size_t)(c + d) * s + c];
  if (d == 0) v.y = 0.0;
  B.band[idx] = v;
}

// ---- stage 2: bulge chasing, one workgroup per instance, one sweep per wave ----------------------
// Lane l works on row rho = l & 15 of a 16 x 16 block and on its columns 4 (l >> 4) .. + 3.
// Reflector of length L from x (x_rho in every lane of row rho): scalars and v_rho.
__device__ __forceinline__ void bulge_reflector(double2 x, int L, int rho, double2& tau, double& beta,
                                                double2& v) {
  const double2 alpha = make_double2(readlane_d(x.x, 0), readlane_d(x.y, 0));
  const double xn2 = sum16(rho >= 1 && rho < L ? x.x * x.x + x.y * x.y : 0.0);
  double2 scal;
  reflector_scalars(alpha, xn2, tau, beta, scal);
  v = rho == 0 ? make_double2(1.0, 0.0) : (rho < L ? cmul(x, scal) : make_double2(0.0, 0.0));
  if (tau.x == 0.0 && tau.y == 0.0) v = rho == 0 ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(1024) void k_bulge(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.x);
  const int n = a.s, T2 = band_T2(n);
  const BandWork B = band_layout(a.work + eig_base_doubles(n, a.kmax), n);
  EigWork W = eig_layout(a.work, n, a.kmax);
  double2* __restrict__ bd = B.band;
  __shared__ int prog[16];   // per wave: (sweep << 12) | steps of that sweep completed
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rho = lane & 15, qd = lane >> 4;
  if (a.tstamp && tid == 0) a.tstamp[0] = wall_clock64();
  if (tid < 16) prog[tid] = tid << 12;
  __syncthreads();
  const int wp = (wave + 15) & 15;
  for (int i = wave; i < n - 1; i += 16) {
    const int Ti = (n - 1 - i + NB - 1) / NB;
    const int Tp = (n - i + NB - 1) / NB;   // steps of sweep i - 1
    double2 vprev = make_double2(0.0, 0.0), taup = make_double2(0.0, 0.0);
    for (int t = 0; t < Ti; ++t) {
      if (i > 0) {
        // step t needs step t + 1 of sweep i - 1 (the rows it shares with this step are final)
        const int need = min(t + 2, Tp);
        while (true) {
          const int pv = __hip_atomic_load(&prog[wp], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          if ((pv >> 12) > i - 1 || (pv & 4095) >= need) break;
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (t == 0 && lane == 0) W.d[i] = bd[(size_t)i * LDB].x;
      const int r0 = i + 1 + t * NB;
      const int L = min(NB, n - r0);
      double2 tau, v;
      double beta;
      if (t == 0) {
        const double2 x = rho < L ? bd[(size_t)i * LDB + 1 + rho] : make_double2(0.0, 0.0);
        bulge_reflector(x, L, rho, tau, beta, v);
        if (lane == 0) {
          bd[(size_t)i * LDB + 1] = make_double2(beta, 0.0);
          W.e[i] = beta;
        }
        if (qd == 0 && rho >= 1 && rho < L) bd[(size_t)i * LDB + 1 + rho] = make_double2(0.0, 0.0);
      } else {
        // block A[r0 + rho, c0 + c] of the rows below the previous step's rows
        const int c0 = r0 - NB;
        double2 b[4], vc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = 4 * qd + k;
          b[k] = rho < L ? bd[(size_t)(c0 + c) * LDB + (NB + rho - c)] : make_double2(0.0, 0.0);
          vc[k] = shfl_z(vprev, c);
        }
        // from the right: B <- B (I - tau' v' v'^H)
        double2 y = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) y = cfma(b[k], vc[k], y);
        y = cadd(y, shfl_xor_z(y, 16));
        y = cadd(y, shfl_xor_z(y, 32));
        const double2 ty = cmul(taup, y);
#pragma unroll
        for (int k = 0; k < 4; ++k) b[k] = cfms(ty, make_double2(vc[k].x, -vc[k].y), b[k]);
        // new reflector from the block's first column, applied from the left
        const double2 x = shfl_z(b[0], rho);
        bulge_reflector(x, L, rho, tau, beta, v);
        const double2 ctv = cmul(make_double2(tau.x, -tau.y), v);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 zk = sum16_z(cjmul(v, b[k]));
          b[k] = cfms(ctv, zk, b[k]);
        }
        if (qd == 0) b[0] = rho == 0 ? make_double2(beta, 0.0) : make_double2(0.0, 0.0);
        if (rho < L) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int c = 4 * qd + k;
            bd[(size_t)(c0 + c) * LDB + (NB + rho - c)] = b[k];
          }
        }
      }
      if (qd == 0) B.V2[((size_t)i * T2 + t) * NB + rho] = v;
      if (lane == 0) B.tau2[(size_t)i * T2 + t] = tau;
      // two-sided update of the diagonal block D = A[r0.., r0..] (L x L): D -= v w^H + w v^H
      {
        double2 dv[4], vk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = 4 * qd + k;
          dv[k] = make_double2(0.0, 0.0);
          if (rho < L && c < L) {
            if (rho >= c) dv[k] = bd[(size_t)(r0 + c) * LDB + (rho - c)];
            else {
              const double2 u = bd[(size_t)(r0 + rho) * LDB + (c - rho)];
              dv[k] = make_double2(u.x, -u.y);
            }
          }
          vk[k] = shfl_z(v, c);
        }
        double2 pr = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) pr = cfma(dv[k], vk[k], pr);
        pr = cadd(pr, shfl_xor_z(pr, 16));
        pr = cadd(pr, shfl_xor_z(pr, 32));
        pr = cmul(tau, pr);
        const double2 m = sum16_z(cjmul(v, pr));
        const double2 mu = cjmul(tau, m);
        const double2 w = csub(pr, cscale(cmul(mu, v), 0.5));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 wk = shfl_z(w, 4 * qd + k);
          dv[k] = cfms(v, make_double2(wk.x, -wk.y), dv[k]);
          dv[k] = cfms(w, make_double2(vk[k].x, -vk[k].y), dv[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int c = 4 * qd + k;
          if (rho < L && c <= rho) {
            double2 val = dv[k];
            if (c == rho) val.y = 0.0;
            bd[(size_t)(r0 + c) * LDB + (rho - c)] = val;
          }
        }
      }
      vprev = v;
      taup = tau;
      if (lane == 0)
        __hip_atomic_store(&prog[wave], (i << 12) | (t + 1), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (lane == 0)
      __hip_atomic_store(&prog[wave], (i + 16) << 12, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  if (a.tstamp && tid == 0) a.tstamp[12] = wall_clock64() - a.tstamp[0];
  if (tid == 0) W.d[n - 1] = bd[(size_t)(n - 1) * LDB].x;
  __syncthreads();
  if (wave == 0) tri_bounds(W, n, a.tstamp, a.status);
}

// ---- back-transformation: u = Q1 Q2 y for BT_NV eigenvectors per workgroup -----------------------
// Stage-2 reflectors sweep by sweep in reverse (the steps of one sweep touch disjoint rows and run
// together, 16 lanes each; the next sweep's reflectors are fetched while the current one is
// applied); then the stage-1 panels in reverse, u <- u - V (T (V^H u)), one eigenvector at a time.
static constexpr int BT_THREADS = 1024;
static constexpr int BT_GROUPS = BT_THREADS / 16;
static constexpr int BT_MAXST = 3;   // steps per 16-lane group and sweep: T2 <= 3 * 64 (s <= 3073)
__global__ __launch_bounds__(BT_THREADS) void k_bt_band(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int n = a.s, kmax = a.kmax, T2 = band_T2(n), npan = band_npan(n);
  const BandWork B = band_layout(a.work + eig_base_doubles(n, kmax), n);
  EigWork W = eig_layout(a.work, n, kmax);
  extern __shared__ double2 u[];   // BT_NV x n
  __shared__ double red[4 * (BT_THREADS / 64)][32];
  __shared__ double2 wv[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t0 = blockIdx.x * BT_NV;
  const int kk = a.kkeep[0];
  for (int idx = tid; idx < BT_NV * n; idx += blockDim.x) {
    const int vv = idx / n, i = idx % n;
    const int t = t0 + vv;
    u[idx] = make_double2(t < kmax && t < kk ? W.Y[(size_t)t * n + i] : 0.0, 0.0);
  }
  const int g = tid >> 4, rho = tid & 15;
  // reflectors of sweep i for this lane: steps g, g + BT_GROUPS, ...
  double2 vn[BT_MAXST], tn[BT_MAXST];
  auto fetch = [&](int i) {
#pragma unroll
    for (int m = 0; m < BT_MAXST; ++m) {
      const int st = g + m * BT_GROUPS;
      const bool ok = i >= 0 && st < T2;
      vn[m] = ok ? B.V2[((size_t)i * T2 + st) * NB + rho] : make_double2(0.0, 0.0);
      tn[m] = ok ? B.tau2[(size_t)i * T2 + st] : make_double2(0.0, 0.0);
    }
  };
  fetch(n - 2);
  __syncthreads();
  const long long tb0 = a.tstamp && tid == 0 && blockIdx.x == 0 ? wall_clock64() : 0;
  for (int i = n - 2; i >= 0; --i) {
    const int Ti = (n - 1 - i + NB - 1) / NB;
    double2 vc[BT_MAXST], tc[BT_MAXST];
#pragma unroll
    for (int m = 0; m < BT_MAXST; ++m) {
      vc[m] = vn[m];
      tc[m] = tn[m];
    }
    fetch(i - 1);
#pragma unroll
    for (int m = 0; m < BT_MAXST; ++m) {
      const int st = g + m * BT_GROUPS;
      if (st >= Ti) break;
      const int r = i + 1 + st * NB + rho;
      const bool ok = r < n;
#pragma unroll
      for (int vv = 0; vv < BT_NV; ++vv) {
        const double2 x = ok ? u[vv * n + r] : make_double2(0.0, 0.0);
        const double2 d = sum16_z(cjmul(vc[m], x));
        if (ok) u[vv * n + r] = cfms(cmul(tc[m], d), vc[m], x);
      }
    }
    __syncthreads();
  }
  const bool row0 = (lane & 15) == 0;
  double* rp = red[wave * 4 + (lane >> 4)];
  const long long tb1 = a.tstamp && tid == 0 && blockIdx.x == 0 ? wall_clock64() : 0;
  if (a.tstamp && tid == 0 && blockIdx.x == 0) a.tstamp[13] = tb1 - tb0;
  for (int p = npan - 1; p >= 0; --p) {
    const int c0 = p * NB, r0 = c0 + NB, h = n - r0, ncol = min(NB, h);
#pragma unroll 1
    for (int vv = 0; vv < BT_NV; ++vv) {
      // w = V^H u over the panel's rows: 16 complex sums, by DPP within 16-lane rows, then LDS
      double2 part[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) part[j] = make_double2(0.0, 0.0);
      for (int r = tid; r < h; r += blockDim.x) {
        const double2 x = u[vv * n + r0 + r];
        const double2* grow = a.G + (size_t)(r0 + r) * n + c0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const double2 ve = j >= ncol || r < j ? make_double2(0.0, 0.0)
                                                : (r == j ? make_double2(1.0, 0.0) : grow[j]);
          part[j] = cadd(part[j], cjmul(ve, x));
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double2 sj = sum16_z(part[j]);
        if (row0) {
          rp[2 * j] = sj.x;
          rp[2 * j + 1] = sj.y;
        }
      }
      __syncthreads();
      if (tid < 32) {
        double acc = 0.0;
        for (int w = 0; w < 4 * (BT_THREADS / 64); ++w) acc += red[w][tid];
        reinterpret_cast<double*>(wv)[tid] = acc;
      }
      __syncthreads();
      // w' = T w (T upper triangular)
      double2 tw = make_double2(0.0, 0.0);
      if (tid < NB) {
        const double2* T = B.T1 + (size_t)p * NB * NB;
        for (int k = tid; k < NB; ++k) tw = cfma(T[tid * NB + k], wv[k], tw);
      }
      __syncthreads();
      if (tid < NB) wv[tid] = tw;
      __syncthreads();
      double2 wr[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) wr[j] = uni2(wv[j]);
      for (int r = tid; r < h; r += blockDim.x) {
        const double2* grow = a.G + (size_t)(r0 + r) * n + c0;
        double2 x = u[vv * n + r0 + r];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const double2 ve = j >= ncol || r < j ? make_double2(0.0, 0.0)
                                                : (r == j ? make_double2(1.0, 0.0) : grow[j]);
          x = cfms(ve, wr[j], x);
        }
        u[vv * n + r0 + r] = x;
      }
      __syncthreads();
    }
  }
  if (a.tstamp && tid == 0 && blockIdx.x == 0) a.tstamp[14] = wall_clock64() - tb1;
  for (int idx = tid; idx < BT_NV * n; idx += blockDim.x) {
    const int vv = idx / n, i = idx % n;
    const int t = t0 + vv;
    if (t < kmax) a.U[(size_t)i * kmax + t] = u[idx];
  }
  if (a.tstamp && tid == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 3), (unsigned long long)wall_clock64());
}

// ---- host -----------------------------------------------------------------------------------------
hipError_t launch_band_reduction(const EigArgs& a, hipStream_t st) {
  const int s = a.s;
  if (s < NB + 2 || s > 2048 + NB) return hipErrorInvalidValue;
  const int npan = band_npan(s);
  const BandWork B0 = band_layout(a.work + eig_base_doubles(s, a.kmax), s);
  for (int p = 0; p < npan; ++p) {
    const int r0 = (p + 1) * NB, h = s - r0;
    // one row per thread up to 1024 rows, two above
    if (h <= 1024) hipLaunchKernelGGL((k_band_panel<1, 1024>), dim3(1, a.batch), dim3(1024), 0, st, a, p);
    else hipLaunchKernelGGL((k_band_panel<2, 1024>), dim3(1, a.batch), dim3(1024), 0, st, a, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_x, dim3((h + XR - 1) / XR, a.batch), dim3(1024), 0, st, a, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_w, dim3((h + WROWS - 1) / WROWS, a.batch), dim3(1024), 0, st, a, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // A22 -= [V | W] [W | V]^H on FP64 matrix cores (accumulating into the trailing matrix)
    GemmArgs g{};
    g.A = B0.Z;
    g.B = B0.Z + NB;
    g.C = a.G + (size_t)r0 * s + r0;
    g.M = h;
    g.N = h;
    g.K = 2 * NB;
    g.offAm = g.offAk = g.offBk = g.offBn = g.offCm = g.offCn = nullptr;
    g.conjA = 0;
    g.conjB = 1;
    g.a_kfast = 1;
    g.b_kfast = 1;
    g.alpha_dev = g.alpha_dev2 = nullptr;
    g.alpha = -1.0;
    g.batch = a.batch;
    g.bsA = g.bsB = g.bsC = a.bs;
    g.bsAlpha = g.bsAlpha2 = 0;
    g.sAm = 3 * NB;
    g.sAk = 1;
    g.sBk = 1;
    g.sBn = 3 * NB;
    g.sCm = s;
    g.sCn = 1;
    g.accum = 1;
    e = launch_gemm(g, DT_C128, DT_C128, DT_C128, DT_C128, GEMM_TILE32, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_band_extract, dim3((unsigned)(((int64_t)s * LDB + 255) / 256), a.batch),
                     dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bulge, dim3(a.batch), dim3(1024), 0, st, a);
  return hipGetLastError();
}

size_t bt_band_lds_bytes(int s) { return (size_t)BT_NV * s * 16; }

hipError_t launch_bt_band(const EigArgs& a, hipStream_t st) {
  const size_t lds = bt_band_lds_bytes(a.s);
  if (lds + 4 * (BT_THREADS / 64) * 32 * 8 + NB * 16 > 160 * 1024 - 512) return hipErrorInvalidValue;
  if (band_T2(a.s) > BT_MAXST * BT_GROUPS) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)k_bt_band, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(k_bt_band, dim3((a.kmax + BT_NV - 1) / BT_NV, a.batch), dim3(BT_THREADS), lds, st,
                     a);
  return hipGetLastError();
}

}  // namespace cbc
