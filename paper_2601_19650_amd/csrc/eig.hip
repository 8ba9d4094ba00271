// FP64 Hermitian eigensolver for the truncation step.
//
// The compression keeps the top-k singular subspace of the joined-leg matrix (Sec. III A: compress the
// joined leg "for example via singular value decomposition"). On the GPU it is reached through the
// FP64 Gram matrix G of that matrix: its top-k eigenvectors span the same subspace and its
// eigenvalues are the squared singular values.
//
// One workgroup (16 waves) solves one G:
//   1. Householder reduction to a real symmetric tridiagonal matrix T = Q^H G Q (reflectors
//      H_j = I - tau_j v_j v_j^H with a real sub-diagonal, as in the standard Hermitian reduction);
//   2. the top-kmax eigenvalues of T by multisection on Sturm counts: a group of lanes evaluates the
//      inertia at several points of the current interval at once;
//   3. eigenvectors of T by inverse iteration with a partially pivoted tridiagonal LU, re-orthogonalised
//      by modified Gram-Schmidt inside clusters of close eigenvalues;
//   4. back-transformation U = Q Y, one group of lanes per eigenvector, reflectors streamed from L2.
#include <float.h>

#include "cbc_internal.h"

namespace cbc {

static constexpr int EIG_THREADS = 1024;

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

// Layout of the scratch buffer (doubles).
struct EigWork {
  double* d;      // s
  double* e;      // s
  double2* tau;   // s
  double2* V;     // s * s   reflector j stored at V[j*s + i], i > j (V[j*s+j+1] = 1)
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
    q = dd[i] - x - ee2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

__global__ __launch_bounds__(EIG_THREADS) void k_eig(EigArgs a) {
  extern __shared__ double smem[];
  const int s = a.s;
  const int kmax = a.kmax;
  double2* vv = reinterpret_cast<double2*>(smem);
  double2* ww = vv + s;
  double* dd = reinterpret_cast<double*>(ww + s);
  double* ee2 = dd + s;
  double* lam = ee2 + s;
  int* cnext = reinterpret_cast<int*>(lam + kmax);
  __shared__ double2 sh_tau, sh_a2;
  __shared__ double sh_lo, sh_hi, sh_pivmin, sh_tnorm;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nwave = blockDim.x >> 6;
  double2* A = a.G;
  EigWork W = eig_layout(a.work, s, kmax);

  // ---- 1. Householder tridiagonalisation ------------------------------------------------------
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
      double2 t = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
      double beta = alpha.x;
      if (!(xn2 == 0.0 && alpha.y == 0.0)) {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        // scal = 1 / (alpha - beta)
        const double ar = alpha.x - beta, ai = alpha.y;
        const double den = ar * ar + ai * ai;
        scal = make_double2(ar / den, -ai / den);
      }
      if (lane == 0) {
        sh_tau = t;
        W.tau[j] = t;
        W.e[j] = beta;
        W.d[j] = A[(size_t)j * s + j].x;
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
    const double2 t = sh_tau;
    if (t.x == 0.0 && t.y == 0.0) continue;
    // p = tau * A_sub v
    for (int r = wave; r < nj; r += nwave) {
      const double2* row = A + (size_t)(j + 1 + r) * s + (j + 1);
      double pr = 0.0, pi = 0.0;
      for (int c = lane; c < nj; c += 64) {
        const double2 x = row[c];
        const double2 v = vv[c];
        pr += x.x * v.x - x.y * v.y;
        pi += x.x * v.y + x.y * v.x;
      }
      pr = wave_sum(pr);
      pi = wave_sum(pi);
      if (lane == 0) ww[r] = cmul(t, make_double2(pr, pi));
    }
    __syncthreads();
    if (wave == 0) {
      double sr = 0.0, si = 0.0;  // w^H v
      for (int i = lane; i < nj; i += 64) {
        const double2 w = ww[i], v = vv[i];
        sr += w.x * v.x + w.y * v.y;
        si += w.x * v.y - w.y * v.x;
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) {
        const double2 q = cmul(t, make_double2(sr, si));
        sh_a2 = make_double2(-0.5 * q.x, -0.5 * q.y);
      }
    }
    __syncthreads();
    const double2 a2 = sh_a2;
    // A_sub -= v w'^H + w' v^H with w' = w + a2 v
    for (int r = wave; r < nj; r += nwave) {
      const double2 vr = vv[r];
      const double2 wr = make_double2(ww[r].x + a2.x * vr.x - a2.y * vr.y,
                                      ww[r].y + a2.x * vr.y + a2.y * vr.x);
      double2* row = A + (size_t)(j + 1 + r) * s + (j + 1);
      for (int c = lane; c < nj; c += 64) {
        const double2 vc = vv[c];
        const double2 wc = make_double2(ww[c].x + a2.x * vc.x - a2.y * vc.y,
                                        ww[c].y + a2.x * vc.y + a2.y * vc.x);
        double2 x = row[c];
        // v_r conj(w_c) + w_r conj(v_c)
        x.x -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
        x.y -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
        row[c] = x;
      }
    }
    __syncthreads();
  }
  if (tid == 0) W.d[s - 1] = A[(size_t)(s - 1) * s + (s - 1)].x;
  __syncthreads();

  // ---- 2. eigenvalues of T: multisection on Sturm counts ----------------------------------------
  for (int i = tid; i < s; i += blockDim.x) {
    dd[i] = W.d[i];
    ee2[i] = i < s - 1 ? W.e[i] * W.e[i] : 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
    for (int i = lane; i < s; i += 64) {
      const double el = i > 0 ? fabs(W.e[i - 1]) : 0.0;
      const double er = i < s - 1 ? fabs(W.e[i]) : 0.0;
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
      sh_lo = lo - pad;
      sh_hi = hi + pad;
      sh_tnorm = tn;
      sh_pivmin = DBL_MIN * fmax(1.0, emax);
    }
  }
  __syncthreads();
  {
    int G = 64;
    while (G > 1 && (EIG_THREADS / G) < kmax) G >>= 1;
    const int ngroups = EIG_THREADS / G;
    const int grp = tid / G;
    const int gl = tid % G;
    const int goff = (lane / G) * G;
    const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const double pivmin = sh_pivmin;
    const double tnorm = sh_tnorm;
    const double width0 = sh_hi - sh_lo;
    const double target = 2.0 * DBL_EPSILON * tnorm + 4.0 * pivmin;
    int rounds = 1;
    {
      double w = width0;
      while (w > target && rounds < 200) { w /= (G + 1); ++rounds; }
    }
    for (int t0 = 0; t0 < kmax; t0 += ngroups) {
      const int t = t0 + grp;
      const bool act = t < kmax;
      const int jidx = s - 1 - (act ? t : 0);  // ascending index of the t-th largest eigenvalue
      double lo = sh_lo, hi = sh_hi;
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
  }
  __syncthreads();

  // ---- 3. eigenvectors of T by inverse iteration ----------------------------------------------
  if (tid == 0) {
    const double ortol = 1e-3 * sh_tnorm;
    int start = 0;
    for (int t = 1; t <= kmax; ++t) {
      if (t == kmax || lam[t - 1] - lam[t] > ortol) {
        for (int u = start; u < t; ++u) cnext[u] = (u == start) ? t : -1;
        start = t;
      }
    }
  }
  __syncthreads();
  for (int cs = tid; cs < kmax; cs += blockDim.x) {
    if (cnext[cs] < 0) continue;
    const int ce = cnext[cs];
    const double tnorm = sh_tnorm;
    const double eps3 = 10.0 * DBL_EPSILON * fmax(tnorm, DBL_MIN);
    double* DL = W.lu + (size_t)cs * 5 * s;
    double* D = DL + s;
    double* DU = D + s;
    double* DU2 = DU + s;
    double* piv = DU2 + s;
    double xprev = 0.0;
    for (int u = cs; u < ce; ++u) {
      double x = lam[u];
      if (u > cs && xprev - x < eps3) x = xprev - eps3;
      xprev = x;
      // factor T - x I = P L U (tridiagonal, partial pivoting)
      for (int i = 0; i < s; ++i) {
        D[i] = dd[i] - x;
        if (i < s - 1) { DL[i] = W.e[i]; DU[i] = W.e[i]; }
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
      double* y = W.Y + (size_t)u * s;
      // deterministic start vector
      for (int i = 0; i < s; ++i) {
        unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)(u * 40503u + 12345u);
        h ^= h >> 13; h *= 0x5bd1e995u; h ^= h >> 15;
        y[i] = 0.5 + double(h & 0xffff) / 65536.0;
      }
      for (int it = 0; it < 3; ++it) {
        // forward: apply P and L^{-1}
        for (int i = 0; i < s - 1; ++i) {
          if (piv[i] == 0.0) {
            y[i + 1] -= DL[i] * y[i];
          } else {
            const double tmp = y[i];
            y[i] = y[i + 1];
            y[i + 1] = tmp - DL[i] * y[i];
          }
        }
        // back: U^{-1}
        y[s - 1] /= D[s - 1];
        if (s > 1) y[s - 2] = (y[s - 2] - DU[s - 2] * y[s - 1]) / D[s - 2];
        for (int i = s - 3; i >= 0; --i) y[i] = (y[i] - DU[i] * y[i + 1] - DU2[i] * y[i + 2]) / D[i];
        // re-orthogonalise against earlier members of the cluster, then normalise
        for (int v = cs; v < u; ++v) {
          const double* yv = W.Y + (size_t)v * s;
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
  __syncthreads();

  // ---- 4. rank selection ------------------------------------------------------------------------
  __shared__ int sh_keep;
  if (tid == 0) {
    int keep = kmax;
    if (a.tol > 0.0) {
      const double cut = a.tol * a.tol * lam[0];
      keep = 0;
      for (int t = 0; t < kmax; ++t) keep += lam[t] > cut;
    }
    if (keep < 1) keep = 1;
    sh_keep = keep;
    a.kkeep[0] = keep;
    a.inv_sqrt_l0[0] = lam[0] > 0.0 ? 1.0 / sqrt(lam[0]) : 1.0;
  }
  for (int t = tid; t < kmax; t += blockDim.x) a.lam[t] = lam[t];
  __syncthreads();
  const int keep = sh_keep;

  // ---- 5. back-transformation U = Q Y -----------------------------------------------------------
  int G2 = 1;
  while (G2 < 64 && G2 * 16 < s) G2 <<= 1;
  const int cols_per_wave = 64 / G2;
  const int gl = lane % G2;
  const int wcol = lane / G2;
  if (G2 * 16 >= s) {
    for (int t = wave * cols_per_wave + wcol; t < kmax; t += nwave * cols_per_wave) {
      double ur[16], ui[16];
      const double* y = W.Y + (size_t)t * s;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = gl + r * G2;
        ur[r] = (i < s) ? y[i] : 0.0;
        ui[r] = 0.0;
      }
      for (int j = s - 2; j >= 0; --j) {
        const double2 tj = W.tau[j];
        if (tj.x == 0.0 && tj.y == 0.0) continue;
        const double2* vj = W.V + (size_t)j * s;
        double dr = 0.0, di = 0.0;  // v^H u over rows > j
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = gl + r * G2;
          if (i > j && i < s) {
            const double2 v = vj[i];
            dr += v.x * ur[r] + v.y * ui[r];
            di += v.x * ui[r] - v.y * ur[r];
          }
        }
        dr = group_sum(dr, G2);
        di = group_sum(di, G2);
        const double2 f = cmul(tj, make_double2(dr, di));
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = gl + r * G2;
          if (i > j && i < s) {
            const double2 v = vj[i];
            ur[r] -= v.x * f.x - v.y * f.y;
            ui[r] -= v.x * f.y + v.y * f.x;
          }
        }
      }
      const bool kept = t < keep;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = gl + r * G2;
        if (i < s) a.U[(size_t)i * kmax + t] = kept ? make_double2(ur[r], ui[r]) : make_double2(0.0, 0.0);
      }
    }
  } else {
    // large s: one wave per column, column kept in global memory
    for (int t = wave; t < kmax; t += nwave) {
      const double* y = W.Y + (size_t)t * s;
      for (int i = lane; i < s; i += 64) a.U[(size_t)i * kmax + t] = make_double2(y[i], 0.0);
      for (int j = s - 2; j >= 0; --j) {
        const double2 tj = W.tau[j];
        if (tj.x == 0.0 && tj.y == 0.0) continue;
        const double2* vj = W.V + (size_t)j * s;
        double dr = 0.0, di = 0.0;
        for (int i = j + 1 + lane; i < s; i += 64) {
          const double2 v = vj[i];
          const double2 u = a.U[(size_t)i * kmax + t];
          dr += v.x * u.x + v.y * u.y;
          di += v.x * u.y - v.y * u.x;
        }
        dr = wave_sum(dr);
        di = wave_sum(di);
        const double2 f = cmul(tj, make_double2(dr, di));
        for (int i = j + 1 + lane; i < s; i += 64) {
          const double2 v = vj[i];
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

hipError_t launch_eig(const EigArgs& a, hipStream_t st) {
  if (a.s <= 0 || a.kmax <= 0 || a.kmax > a.s) return hipErrorInvalidValue;
  const size_t lds = (size_t)a.s * (2 * sizeof(double2) + 2 * sizeof(double)) +
                     (size_t)a.kmax * (sizeof(double) + sizeof(int)) + 64;
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eig, dim3(1), dim3(EIG_THREADS), lds, st, a);
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
