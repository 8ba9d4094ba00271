// FP64 Hermitian eigensolver for the truncation step.
//
// The compression keeps the top-k singular subspace of the joined-leg matrix (Sec. III A: compress the
// joined leg "for example via singular value decomposition"). On the GPU it is reached through the
// FP64 Gram matrix G of that matrix: its top-k eigenvectors span the same subspace and its
// eigenvalues are the squared singular values.
//
// One workgroup (16 waves) solves one G:
//   1. Householder reduction to a real symmetric tridiagonal T = Q^H G Q (reflectors
//      H_j = I - tau_j v_j v_j^H, real sub-diagonal). For s <= EIG_LDS_MAX the packed lower triangle
//      lives in LDS; larger matrices are reduced in place in global memory (L2 resident). The
//      Hermitian matrix-vector product is done by groups of 8 lanes per row and the dot product w^H v
//      is folded into it, so a step costs three workgroup barriers.
//   2. the top-kmax eigenvalues of T by multisection on Sturm counts: a group of lanes evaluates the
//      inertia at several points of the current interval at once;
//   3. eigenvectors of T: a twisted factorisation T - lambda I = N_r Delta N_r^T per eigenvalue (one
//      lane each, no memory-carried dependency chains); eigenvalues closer than 1e-3 ||T|| to a
//      neighbour are handled together by inverse iteration with modified Gram-Schmidt;
//   4. back-transformation U = Q Y, one group of lanes per eigenvector with the column in registers.
#include <float.h>

#include "cbc_internal.h"

namespace cbc {

static constexpr int EIG_THREADS = 1024;
static constexpr int EIG_LDS_MAX = 128;   // largest s whose packed triangle stays in LDS
static constexpr int RG = 8;              // lanes per row group in the matrix-vector product

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double group_sum(double v, int g) {
  for (int o = g >> 1; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ int tri(int r) { return r * (r + 1) / 2; }
// a / b through the hardware reciprocal refined by one Newton step (a few ulp; used only in the Sturm
// count and the twisted factorisation, whose callers guard b away from zero).
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}

// Layout of the scratch buffer (doubles).
struct EigWork {
  double* d;      // s
  double* e;      // s
  double2* tau;   // s
  double2* V;     // s * s   (global path) reflector j at V[j*s + i], i > j, V[j*s+j+1] = 1
  double* Y;      // kmax * s   eigenvector t of T at Y[t*s + i]
  double* lu;     // kmax * 5 * s
};
__host__ __device__ inline EigWork eig_layout(double* w, int s, int kmax) {
  EigWork L;
  L.d = w;
  L.e = w + s;
  L.tau = reinterpret_cast<double2*>(w + 2 * (size_t)s);
  L.V = reinterpret_cast<double2*>(w + 4 * (size_t)s);
  L.Y = w + 4 * (size_t)s + 2 * (size_t)s * s;
  L.lu = L.Y + (size_t)kmax * s;
  return L;
}
size_t eig_work_doubles(int s, int kmax) {
  return 4 * (size_t)s + 2 * (size_t)s * s + (size_t)kmax * s + 5 * (size_t)kmax * s + 64;
}

__device__ int sturm_count(const double* dd, const double* ee2, int s, double x, double pivmin) {
  double q = dd[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  for (int i = 1; i < s; ++i) {
    q = dd[i] - x - qdiv(ee2[i - 1], q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

struct Shared {
  double2 tau, a2;
  double lo, hi, pivmin, tnorm;
  double dotr, doti;
  int keep;
};

// Householder vector of column j from x = A[j+1.., j]; called by wave 0 only.
// Writes tau, beta into sh/W and returns the scaling 1/(alpha - beta) applied to x[1..].
__device__ inline double2 householder(double2 alpha, double xn2, int j, double a_jj, Shared& sh,
                                      EigWork& W, int lane) {
  double2 t = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
  double beta = alpha.x;
  if (!(xn2 == 0.0 && alpha.y == 0.0)) {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double ar = alpha.x - beta, ai = alpha.y;
    const double den = ar * ar + ai * ai;
    scal = make_double2(ar / den, -ai / den);
  }
  if (lane == 0) {
    sh.tau = t;
    W.tau[j] = t;
    W.e[j] = beta;
    W.d[j] = a_jj;
    sh.dotr = 0.0;
    sh.doti = 0.0;
  }
  return scal;
}

// ---- reduction with the packed lower triangle in LDS -------------------------------------------
__device__ void tridiag_lds(double2* P, double2* vv, double2* ww, const double2* G, int s, Shared& sh,
                            EigWork& W) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nthr = blockDim.x;
  for (int idx = tid; idx < tri(s); idx += nthr) {
    // row r of the packed triangle from G (row-major, both triangles valid)
    int r = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while (tri(r + 1) <= idx) ++r;
    while (tri(r) > idx) --r;
    const int c = idx - tri(r);
    P[idx] = G[(size_t)r * s + c];
  }
  __syncthreads();
  const int grp = tid / RG, gl = tid % RG, ngrp = nthr / RG;
  for (int j = 0; j < s - 1; ++j) {
    const int nj = s - j - 1;
    if (wave == 0) {
      const double2 alpha = P[tri(j + 1) + j];
      double xn2 = 0.0;
      for (int i = j + 2 + lane; i < s; i += 64) {
        const double2 x = P[tri(i) + j];
        xn2 += x.x * x.x + x.y * x.y;
      }
      xn2 = wave_sum(xn2);
      const double2 scal = householder(alpha, xn2, j, P[tri(j) + j].x, sh, W, lane);
      if (lane == 0) vv[0] = make_double2(1.0, 0.0);
      for (int i = 1 + lane; i < nj; i += 64) {
        const double2 v = cmul(P[tri(j + 1 + i) + j], scal);
        vv[i] = v;
        P[tri(j + 1 + i) + j] = v;   // reflector kept below the sub-diagonal for the back-transform
      }
    }
    __syncthreads();
    const double2 t = sh.tau;
    if (t.x == 0.0 && t.y == 0.0) continue;
    // p = tau A_sub v by row groups; w = p; partial w^H v accumulated in LDS
    double dacc_r = 0.0, dacc_i = 0.0;
    for (int r = grp; r < nj; r += ngrp) {
      const int R = j + 1 + r;
      double pr = 0.0, pi = 0.0;
      for (int c = gl; c < nj; c += RG) {
        const int C = j + 1 + c;
        const double2 a = (c <= r) ? P[tri(R) + C] : cconj(P[tri(C) + R]);
        const double2 v = vv[c];
        pr += a.x * v.x - a.y * v.y;
        pi += a.x * v.y + a.y * v.x;
      }
      pr = group_sum(pr, RG);
      pi = group_sum(pi, RG);
      if (gl == 0) {
        const double2 w = cmul(t, make_double2(pr, pi));
        ww[r] = w;
        const double2 v = vv[r];
        dacc_r += w.x * v.x + w.y * v.y;
        dacc_i += w.x * v.y - w.y * v.x;
      }
    }
    // w^H v: reduce the row-group leaders' partials across the wave, one LDS atomic per wave
    dacc_r = wave_sum(dacc_r);
    dacc_i = wave_sum(dacc_i);
    if (lane == 0) {
      atomicAdd(&sh.dotr, dacc_r);
      atomicAdd(&sh.doti, dacc_i);
    }
    __syncthreads();
    const double2 q = cmul(t, make_double2(sh.dotr, sh.doti));
    const double2 a2 = make_double2(-0.5 * q.x, -0.5 * q.y);
    // lower-triangle update A_sub -= v w'^H + w' v^H, w' = w + a2 v
    for (int r = grp; r < nj; r += ngrp) {
      const int R = j + 1 + r;
      const double2 vr = vv[r];
      const double2 wr = make_double2(ww[r].x + a2.x * vr.x - a2.y * vr.y,
                                      ww[r].y + a2.x * vr.y + a2.y * vr.x);
      for (int c = gl; c <= r; c += RG) {
        const double2 vc = vv[c];
        const double2 wc = make_double2(ww[c].x + a2.x * vc.x - a2.y * vc.y,
                                        ww[c].y + a2.x * vc.y + a2.y * vc.x);
        double2 x = P[tri(R) + j + 1 + c];
        x.x -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
        x.y -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
        P[tri(R) + j + 1 + c] = x;
      }
    }
    __syncthreads();
  }
  if (tid == 0) W.d[s - 1] = P[tri(s - 1) + s - 1].x;
  __syncthreads();
}

// ---- reduction in global memory (both triangles kept) -------------------------------------------
__device__ void tridiag_global(double2* A, double2* vv, double2* ww, int s, Shared& sh, EigWork& W) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nthr = blockDim.x;
  const int grp = tid / RG, gl = tid % RG, ngrp = nthr / RG;
  for (int j = 0; j < s - 1; ++j) {
    const int nj = s - j - 1;
    if (wave == 0) {
      const double2 alpha = A[(size_t)(j + 1) * s + j];
      double xn2 = 0.0;
      for (int i = j + 2 + lane; i < s; i += 64) {
        const double2 x = A[(size_t)i * s + j];
        xn2 += x.x * x.x + x.y * x.y;
      }
      xn2 = wave_sum(xn2);
      const double2 scal = householder(alpha, xn2, j, A[(size_t)j * s + j].x, sh, W, lane);
      if (lane == 0) {
        vv[0] = make_double2(1.0, 0.0);
        W.V[(size_t)j * s + j + 1] = make_double2(1.0, 0.0);
      }
      for (int i = 1 + lane; i < nj; i += 64) {
        const double2 v = cmul(A[(size_t)(j + 1 + i) * s + j], scal);
        vv[i] = v;
        W.V[(size_t)j * s + j + 1 + i] = v;
      }
    }
    __syncthreads();
    const double2 t = sh.tau;
    if (t.x == 0.0 && t.y == 0.0) continue;
    double dacc_r = 0.0, dacc_i = 0.0;
    for (int r = grp; r < nj; r += ngrp) {
      const double2* row = A + (size_t)(j + 1 + r) * s + (j + 1);
      double pr = 0.0, pi = 0.0;
      for (int c = gl; c < nj; c += RG) {
        const double2 a = row[c];
        const double2 v = vv[c];
        pr += a.x * v.x - a.y * v.y;
        pi += a.x * v.y + a.y * v.x;
      }
      pr = group_sum(pr, RG);
      pi = group_sum(pi, RG);
      if (gl == 0) {
        const double2 w = cmul(t, make_double2(pr, pi));
        ww[r] = w;
        const double2 v = vv[r];
        dacc_r += w.x * v.x + w.y * v.y;
        dacc_i += w.x * v.y - w.y * v.x;
      }
    }
    // w^H v: reduce the row-group leaders' partials across the wave, one LDS atomic per wave
    dacc_r = wave_sum(dacc_r);
    dacc_i = wave_sum(dacc_i);
    if (lane == 0) {
      atomicAdd(&sh.dotr, dacc_r);
      atomicAdd(&sh.doti, dacc_i);
    }
    __syncthreads();
    const double2 q = cmul(t, make_double2(sh.dotr, sh.doti));
    const double2 a2 = make_double2(-0.5 * q.x, -0.5 * q.y);
    for (int r = wave; r < nj; r += nthr / 64) {
      const double2 vr = vv[r];
      const double2 wr = make_double2(ww[r].x + a2.x * vr.x - a2.y * vr.y,
                                      ww[r].y + a2.x * vr.y + a2.y * vr.x);
      double2* row = A + (size_t)(j + 1 + r) * s + (j + 1);
      for (int c = lane; c < nj; c += 64) {
        const double2 vc = vv[c];
        const double2 wc = make_double2(ww[c].x + a2.x * vc.x - a2.y * vc.y,
                                        ww[c].y + a2.x * vc.y + a2.y * vc.x);
        double2 x = row[c];
        x.x -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
        x.y -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
        row[c] = x;
      }
    }
    __syncthreads();
  }
  if (tid == 0) W.d[s - 1] = A[(size_t)(s - 1) * s + (s - 1)].x;
  __syncthreads();
}

// ---- eigenvalues: multisection --------------------------------------------------------------------
__device__ void eigenvalues(const double* dd, const double* ee2, const double* e, int s, int kmax,
                            double* lam, Shared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (wave == 0) {
    double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
    for (int i = lane; i < s; i += 64) {
      const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
      const double er = i < s - 1 ? fabs(e[i]) : 0.0;
      lo = fmin(lo, dd[i] - el - er);
      hi = fmax(hi, dd[i] + el + er);
      emax = fmax(emax, ee2[i]);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    emax = wave_max(emax);
    if (lane == 0) {
      const double tn = fmax(fabs(lo), fabs(hi));
      const double pad = 2.0 * DBL_EPSILON * tn * s + DBL_MIN;
      sh.lo = lo - pad;
      sh.hi = hi + pad;
      sh.tnorm = tn;
      sh.pivmin = DBL_MIN * fmax(1.0, emax);
    }
  }
  __syncthreads();
  int G = 64;
  while (G > 1 && (EIG_THREADS / G) < kmax) G >>= 1;
  const int ngroups = EIG_THREADS / G;
  const int grp = tid / G;
  const int gl = tid % G;
  const int goff = (lane / G) * G;
  const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  const double pivmin = sh.pivmin;
  const double target = 2.0 * DBL_EPSILON * sh.tnorm + 4.0 * pivmin;
  int rounds = 1;
  {
    double w = sh.hi - sh.lo;
    while (w > target && rounds < 200) { w /= (G + 1); ++rounds; }
  }
  for (int t0 = 0; t0 < kmax; t0 += ngroups) {
    const int t = t0 + grp;
    const bool act = t < kmax;
    const int jidx = s - 1 - (act ? t : 0);
    double lo = sh.lo, hi = sh.hi;
    for (int rd = 0; rd < rounds; ++rd) {
      const double x = lo + (hi - lo) * double(gl + 1) / double(G + 1);
      const int c = sturm_count(dd, ee2, s, x, pivmin);
      const unsigned long long m = __ballot(c <= jidx);
      const int b = __popcll((m >> goff) & gmask);
      const double xlo = lo + (hi - lo) * double(b) / double(G + 1);
      const double xhi = lo + (hi - lo) * double(b + 1) / double(G + 1);
      lo = xlo;
      hi = xhi;
    }
    if (act && gl == 0) lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();
}

// ---- eigenvectors of T ----------------------------------------------------------------------------
// Twisted factorisation for an isolated eigenvalue x: y gets the unit eigenvector.
__device__ void twisted_vector(const double* dd, const double* e, int s, double x, double pivmin,
                               double* y, double* lp, double* dp, double* um) {
  double d = dd[0] - x;
  dp[0] = d;
  for (int i = 0; i < s - 1; ++i) {
    if (fabs(d) < pivmin) d = d < 0.0 ? -pivmin : pivmin;
    const double l = qdiv(e[i], d);
    lp[i] = l;
    d = dd[i + 1] - x - l * e[i];
    dp[i + 1] = d;
  }
  // backward factorisation and twist index r = argmin |gamma_r|
  double dm = dd[s - 1] - x;
  int r = s - 1;
  double gbest = fabs(dp[s - 1]);
  for (int i = s - 2; i >= 0; --i) {
    if (fabs(dm) < pivmin) dm = dm < 0.0 ? -pivmin : pivmin;
    const double u = qdiv(e[i], dm);
    um[i] = u;
    dm = dd[i] - x - u * e[i];
    const double g = fabs(dp[i] + dm - (dd[i] - x));
    if (g < gbest) { gbest = g; r = i; }
  }
  double z = 1.0, nrm = 1.0;
  y[r] = 1.0;
  for (int i = r - 1; i >= 0; --i) {
    z = -lp[i] * z;
    y[i] = z;
    nrm += z * z;
  }
  z = 1.0;
  for (int i = r; i < s - 1; ++i) {
    z = -um[i] * z;
    y[i + 1] = z;
    nrm += z * z;
  }
  const double inv = 1.0 / sqrt(nrm);
  for (int i = 0; i < s; ++i) y[i] *= inv;
}

// Inverse iteration for the members [cs, ce) of a cluster, re-orthogonalised within the cluster.
__device__ void cluster_vectors(const double* dd, const double* e, int s, const double* lam, int cs,
                                int ce, double tnorm, double* Y, double* scratch) {
  const double eps3 = 10.0 * DBL_EPSILON * fmax(tnorm, DBL_MIN);
  double* DL = scratch;
  double* D = DL + s;
  double* DU = D + s;
  double* DU2 = DU + s;
  double* piv = DU2 + s;
  double xprev = 0.0;
  for (int u = cs; u < ce; ++u) {
    double x = lam[u];
    if (u > cs && xprev - x < eps3) x = xprev - eps3;
    xprev = x;
    for (int i = 0; i < s; ++i) {
      D[i] = dd[i] - x;
      if (i < s - 1) { DL[i] = e[i]; DU[i] = e[i]; }
      DU2[i] = 0.0;
      piv[i] = 0.0;
    }
    for (int i = 0; i < s - 1; ++i) {
      if (fabs(D[i]) >= fabs(DL[i])) {
        if (D[i] == 0.0) D[i] = eps3;
        const double f = DL[i] / D[i];
        DL[i] = f;
        D[i + 1] -= f * DU[i];
      } else {
        const double f = D[i] / DL[i];
        D[i] = DL[i];
        DL[i] = f;
        const double tmp = DU[i];
        DU[i] = D[i + 1];
        D[i + 1] = tmp - f * D[i + 1];
        if (i < s - 2) {
          DU2[i] = DU[i + 1];
          DU[i + 1] = -f * DU[i + 1];
        }
        piv[i] = 1.0;
      }
    }
    if (D[s - 1] == 0.0) D[s - 1] = eps3;
    double* y = Y + (size_t)u * s;
    for (int i = 0; i < s; ++i) {
      unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)(u * 40503u + 12345u);
      h ^= h >> 13; h *= 0x5bd1e995u; h ^= h >> 15;
      y[i] = 0.5 + double(h & 0xffff) / 65536.0;
    }
    for (int it = 0; it < 3; ++it) {
      for (int i = 0; i < s - 1; ++i) {
        if (piv[i] == 0.0) {
          y[i + 1] -= DL[i] * y[i];
        } else {
          const double tmp = y[i];
          y[i] = y[i + 1];
          y[i + 1] = tmp - DL[i] * y[i];
        }
      }
      y[s - 1] /= D[s - 1];
      if (s > 1) y[s - 2] = (y[s - 2] - DU[s - 2] * y[s - 1]) / D[s - 2];
      for (int i = s - 3; i >= 0; --i) y[i] = (y[i] - DU[i] * y[i + 1] - DU2[i] * y[i + 2]) / D[i];
      for (int v = cs; v < u; ++v) {
        const double* yv = Y + (size_t)v * s;
        double dot = 0.0;
        for (int i = 0; i < s; ++i) dot += yv[i] * y[i];
        for (int i = 0; i < s; ++i) y[i] -= dot * yv[i];
      }
      double nrm = 0.0, mx = 0.0;
      for (int i = 0; i < s; ++i) mx = fmax(mx, fabs(y[i]));
      if (mx == 0.0) { y[u % s] = 1.0; mx = 1.0; }
      for (int i = 0; i < s; ++i) { y[i] /= mx; nrm += y[i] * y[i]; }
      const double inv = 1.0 / sqrt(nrm);
      for (int i = 0; i < s; ++i) y[i] *= inv;
    }
  }
}

__device__ void eigenvectors(const double* dd, const double* e, int s, int kmax, const double* lam,
                             int* cnext, Shared& sh, EigWork& W) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    // clusters of non-negligible eigenvalues closer than 1e-3 ||T|| (negligible ones, at the
    // rounding level of ||T||, are computed one by one: they carry no weight)
    const double ortol = 1e-3 * sh.tnorm;
    const double tiny = 64.0 * DBL_EPSILON * sh.tnorm;
    int start = 0;
    for (int t = 1; t <= kmax; ++t) {
      const bool split = t == kmax || lam[t - 1] - lam[t] > ortol || lam[t] <= tiny;
      if (split) {
        for (int u = start; u < t; ++u) cnext[u] = (u == start) ? t : -1;
        start = t;
      }
    }
  }
  __syncthreads();
  for (int cs = tid; cs < kmax; cs += blockDim.x) {
    const int ce = cnext[cs];
    if (ce < 0) continue;
    double* scratch = W.lu + (size_t)cs * 5 * s;
    if (ce == cs + 1) {
      twisted_vector(dd, e, s, lam[cs], sh.pivmin, W.Y + (size_t)cs * s, scratch, scratch + s,
                     scratch + 2 * s);
    } else {
      cluster_vectors(dd, e, s, lam, cs, ce, sh.tnorm, W.Y, scratch);
    }
  }
  __syncthreads();
}

// ---- rank selection and back-transformation -------------------------------------------------------
__device__ void select_rank(const EigArgs& a, const double* lam, int kmax, Shared& sh) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    int keep = kmax;
    if (a.tol > 0.0) {
      const double cut = a.tol * a.tol * lam[0];
      keep = 0;
      for (int t = 0; t < kmax; ++t) keep += lam[t] > cut;
    }
    if (keep < 1) keep = 1;
    sh.keep = keep;
    a.kkeep[0] = keep;
    a.inv_sqrt_l0[0] = lam[0] > 0.0 ? 1.0 / sqrt(lam[0]) : 1.0;
  }
  for (int t = tid; t < kmax; t += blockDim.x) a.lam[t] = lam[t];
  __syncthreads();
}

// VFn(j, i) returns component i (> j) of reflector j.
template <typename VFn>
__device__ void back_transform(const EigArgs& a, int s, int kmax, int keep, EigWork& W,
                               const double2* taus, VFn vget) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  constexpr int RR = 8;   // rows of the column held by each lane
  int G2 = 1;
  while (G2 < 64 && G2 * RR < s) G2 <<= 1;
  const int cols_per_wave = 64 / G2;
  const int gl = lane % G2;
  const int wcol = lane / G2;
  if (G2 * RR >= s) {
    for (int t = wave * cols_per_wave + wcol; t < kmax; t += nwave * cols_per_wave) {
      double ur[RR], ui[RR];
      const double* y = W.Y + (size_t)t * s;
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        const int i = gl + r * G2;
        ur[r] = (i < s) ? y[i] : 0.0;
        ui[r] = 0.0;
      }
      for (int j = s - 2; j >= 0; --j) {
        const double2 tj = taus[j];
        if (tj.x == 0.0 && tj.y == 0.0) continue;
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          const int i = gl + r * G2;
          if (i > j && i < s) {
            const double2 v = vget(j, i);
            dr += v.x * ur[r] + v.y * ui[r];
            di += v.x * ui[r] - v.y * ur[r];
          }
        }
        dr = group_sum(dr, G2);
        di = group_sum(di, G2);
        const double2 f = cmul(tj, make_double2(dr, di));
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          const int i = gl + r * G2;
          if (i > j && i < s) {
            const double2 v = vget(j, i);
            ur[r] -= v.x * f.x - v.y * f.y;
            ui[r] -= v.x * f.y + v.y * f.x;
          }
        }
      }
      const bool kept = t < keep;
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        const int i = gl + r * G2;
        if (i < s) a.U[(size_t)i * kmax + t] = kept ? make_double2(ur[r], ui[r]) : make_double2(0.0, 0.0);
      }
    }
  } else {
    for (int t = wave; t < kmax; t += nwave) {
      const double* y = W.Y + (size_t)t * s;
      for (int i = lane; i < s; i += 64) a.U[(size_t)i * kmax + t] = make_double2(y[i], 0.0);
      for (int j = s - 2; j >= 0; --j) {
        const double2 tj = taus[j];
        if (tj.x == 0.0 && tj.y == 0.0) continue;
        double dr = 0.0, di = 0.0;
        for (int i = j + 1 + lane; i < s; i += 64) {
          const double2 v = vget(j, i);
          const double2 u = a.U[(size_t)i * kmax + t];
          dr += v.x * u.x + v.y * u.y;
          di += v.x * u.y - v.y * u.x;
        }
        dr = wave_sum(dr);
        di = wave_sum(di);
        const double2 f = cmul(tj, make_double2(dr, di));
        for (int i = j + 1 + lane; i < s; i += 64) {
          const double2 v = vget(j, i);
          double2 u = a.U[(size_t)i * kmax + t];
          u.x -= v.x * f.x - v.y * f.y;
          u.y -= v.x * f.y + v.y * f.x;
          a.U[(size_t)i * kmax + t] = u;
        }
      }
      if (t >= keep)
        for (int i = lane; i < s; i += 64) a.U[(size_t)i * kmax + t] = make_double2(0.0, 0.0);
    }
  }
}

// LDS layout: [packed triangle (lds path only)] vv ww (s complex each) dd ee2 e (s doubles each)
// lam (kmax doubles) tau (s complex) cnext (kmax ints)
template <bool IN_LDS>
__global__ __launch_bounds__(EIG_THREADS) void k_eig(EigArgs a) {
  extern __shared__ double smem[];
  __shared__ Shared sh;
  const int s = a.s, kmax = a.kmax, tid = threadIdx.x;
  double2* P = reinterpret_cast<double2*>(smem);
  double2* vv = IN_LDS ? P + tri(s) : P;
  double2* ww = vv + s;
  double* dd = reinterpret_cast<double*>(ww + s);
  double* ee2 = dd + s;
  double* el = ee2 + s;
  double* lam = el + s;
  double2* taus = reinterpret_cast<double2*>(lam + kmax);
  int* cnext = reinterpret_cast<int*>(taus + s);
  EigWork W = eig_layout(a.work, s, kmax);
  long long* ts = a.tstamp;
  if (tid == 0) {
    sh.dotr = 0.0;
    sh.doti = 0.0;
    if (ts) ts[0] = wall_clock64();
  }
  __syncthreads();
  if (IN_LDS) tridiag_lds(P, vv, ww, a.G, s, sh, W);
  else tridiag_global(a.G, vv, ww, s, sh, W);
  if (ts && tid == 0) ts[1] = wall_clock64();
  for (int i = tid; i < s; i += blockDim.x) {
    dd[i] = W.d[i];
    el[i] = i < s - 1 ? W.e[i] : 0.0;
    ee2[i] = el[i] * el[i];
    taus[i] = i < s - 1 ? W.tau[i] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  eigenvalues(dd, ee2, el, s, kmax, lam, sh);
  if (ts && tid == 0) ts[2] = wall_clock64();
  eigenvectors(dd, el, s, kmax, lam, cnext, sh, W);
  if (ts && tid == 0) ts[3] = wall_clock64();
  select_rank(a, lam, kmax, sh);
  const int keep = sh.keep;
  if (IN_LDS) {
    back_transform(a, s, kmax, keep, W, taus, [&](int j, int i) {
      return i == j + 1 ? make_double2(1.0, 0.0) : P[tri(i) + j];
    });
  } else {
    const double2* V = W.V;
    back_transform(a, s, kmax, keep, W, taus, [&](int j, int i) { return V[(size_t)j * s + i]; });
  }
  __syncthreads();
  if (ts && tid == 0) ts[4] = wall_clock64();
}

size_t eig_lds_bytes(int s, int kmax, bool in_lds) {
  return (in_lds ? (size_t)16 * (s * (size_t)(s + 1) / 2) : 0) + (size_t)s * (3 * 16 + 3 * 8) +
         (size_t)kmax * (8 + 4) + 64;
}

hipError_t launch_eig(const EigArgs& a, hipStream_t st) {
  if (a.s <= 0 || a.kmax <= 0 || a.kmax > a.s) return hipErrorInvalidValue;
  const bool in_lds = a.s <= EIG_LDS_MAX;
  const size_t lds = eig_lds_bytes(a.s, a.kmax, in_lds);
  if (lds > 160 * 1024 - 512) return hipErrorInvalidValue;
  if (in_lds) {
    (void)hipFuncSetAttribute((const void*)k_eig<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k_eig<true>, dim3(1), dim3(EIG_THREADS), lds, st, a);
  } else {
    (void)hipFuncSetAttribute((const void*)k_eig<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k_eig<false>, dim3(1), dim3(EIG_THREADS), lds, st, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
__global__ void k_form_l_nside(const double2* V, const double* lam, const int* kkeep, int n,
                               int kmax, void* L, int tl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)kmax * n) return;
  const int j = (int)(idx / n);
  const int c = (int)(idx % n);
  double2 out = make_double2(0.0, 0.0);
  if (j < kkeep[0] && lam[0] > 0.0) {
    const double f = sqrt(fmax(lam[j], 0.0) / lam[0]);
    const double2 v = V[(size_t)c * kmax + j];
    out = make_double2(f * v.x, -f * v.y);
  }
  if (tl == DT_C128) reinterpret_cast<double2*>(L)[idx] = out;
  else reinterpret_cast<float2*>(L)[idx] = make_float2((float)out.x, (float)out.y);
}

hipError_t launch_form_l_nside(const double2* V, const double* lam, const int* kkeep, int n,
                               int kmax, void* L, DType tl, hipStream_t st) {
  const int64_t tot = (int64_t)kmax * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_form_l_nside, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, V, lam,
                     kkeep, n, kmax, L, (int)tl);
  return hipGetLastError();
}

}  // namespace cbc
