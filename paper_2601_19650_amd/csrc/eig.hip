// FP64 Hermitian eigensolver for the truncation step.
//
// The compression keeps the top-k singular subspace of the joined-leg matrix (Sec. III A: compress the
// joined leg "for example via singular value decomposition"). On the GPU it is reached through the
// FP64 Gram matrix G of that matrix: its top-k eigenvectors span the same subspace and its
// eigenvalues are the squared singular values.
//
// Three launches solve one G:
//   1. k_tridiag, one workgroup (16 waves): Householder reduction to a real symmetric tridiagonal
//      T = Q^H G Q (reflectors H_j = I - tau_j v_j v_j^H, real sub-diagonal). For s <= EIG_LDS_MAX the
//      packed lower triangle lives in LDS; larger matrices are reduced in place in global memory (L2
//      resident). The Hermitian matrix-vector product is done by groups of 8 lanes per row, its
//      reductions use DPP lane moves, and the dot product w^H v is folded into it (per-wave partials
//      added in a fixed order, so results are bitwise reproducible), so a step costs three
//      workgroup barriers. This is the only sequential part.
//   2. k_eigvals, one wave per eigenvalue over many workgroups: the top-kmax eigenvalues of T by
//      multisection on Sturm counts (64 points of the current interval per round).
//   3. k_eigvecs, one wave per eigenpair over many workgroups: the eigenvector of T by a twisted
//      factorisation T - lambda I = N_r Delta N_r^T (eigenvalues closer than 1e-3 ||T|| to a neighbour
//      are handled together, by the wave of the first one, with inverse iteration and modified
//      Gram-Schmidt), then the back-transformation u = Q y with the reflectors streamed from L2.
#include <float.h>

#include "cbc_internal.h"

namespace cbc {

static constexpr int EIG_THREADS = 1024;
static constexpr int EIG_LDS_MAX = 128;   // largest s whose packed triangle stays in LDS
static constexpr int RG = 8;              // lanes per row group in the matrix-vector product

// ---- cross-lane reductions ---------------------------------------------------------------------
// DPP lane moves (quad permutes and row mirrors) are single-cycle VALU operations; ds_bpermute
// (__shfl_xor) goes through the LDS crossbar. A double is moved as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}
// sum over aligned groups of 8 lanes, result in every lane of the group
__device__ __forceinline__ double sum8(double v) {
  v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);   // row_half_mirror
  return v;
}
// sum over aligned rows of 16 lanes, result in every lane of the row
__device__ __forceinline__ double sum16(double v) {
  v = sum8(v);
  v += dpp<0x140>(v);   // row_mirror
  return v;
}
// sum over the wave, result in every lane
__device__ __forceinline__ double wave_sum(double v) {
  v = sum16(v);
  const int lo = __double2loint(v), hi = __double2hiint(v);
  double t = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    t += __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * r), __builtin_amdgcn_readlane(lo, 16 * r));
  return t;
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
  double* bounds; // 8: lo, hi, tnorm, pivmin
  double2* V;     // s * s   reflector j at V[j*s + i], i > j, V[j*s+j+1] = 1
  double* Y;      // kmax * s   cluster eigenvectors of T at Y[t*s + i]
  double* lu;     // kmax * 5 * s
};
__host__ __device__ inline EigWork eig_layout(double* w, int s, int kmax) {
  EigWork L;
  L.d = w;
  L.e = w + s;
  L.tau = reinterpret_cast<double2*>(w + 2 * (size_t)s);
  L.bounds = w + 4 * (size_t)s;
  L.V = reinterpret_cast<double2*>(w + 4 * (size_t)s + 8);
  L.Y = w + 4 * (size_t)s + 8 + 2 * (size_t)s * s;
  L.lu = L.Y + (size_t)kmax * s;
  return L;
}
size_t eig_work_doubles(int s, int kmax) {
  return 4 * (size_t)s + 8 + 2 * (size_t)s * s + (size_t)kmax * s + 5 * (size_t)kmax * s + 64;
}

// EigArgs of instance b (every pointer except the time stamps advances by a.bs bytes)
__device__ inline EigArgs eig_inst(const EigArgs& a0, int b) {
  EigArgs a = a0;
  a.G = inst_ptr(a0.G, a0.bs, b);
  a.U = inst_ptr(a0.U, a0.bs, b);
  a.lam = inst_ptr(a0.lam, a0.bs, b);
  a.kkeep = inst_ptr(a0.kkeep, a0.bs, b);
  a.inv_sqrt_l0 = inst_ptr(a0.inv_sqrt_l0, a0.bs, b);
  a.work = inst_ptr(a0.work, a0.bs, b);
  return a;
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

struct TriShared {
  double2 tau;
  double dotr, doti;
  double2 part[EIG_THREADS / 64];   // per-wave partial sums of w^H v, added in a fixed order
};

// Householder vector of column j from x = A[j+1.., j]; wave 0. Returns the scaling 1/(alpha - beta)
// that maps x[1..] to the reflector.
__device__ inline double2 householder(double2 alpha, double xn2, int j, double a_jj, TriShared& sh,
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

// Hermitian matrix-vector product row p_r = tau sum_c A[r][c] v[c] for one row group, plus the
// row's contribution to w^H v.
template <typename AFn>
__device__ __forceinline__ void matvec_row(int r, int nj, int gl, const double2* vv, double2 t,
                                           AFn aget, double2* ww, double& dr_acc, double& di_acc) {
  double pr = 0.0, pi = 0.0;
  for (int c = gl; c < nj; c += RG) {
    const double2 a = aget(r, c);
    const double2 v = vv[c];
    pr += a.x * v.x - a.y * v.y;
    pi += a.x * v.y + a.y * v.x;
  }
  pr = sum8(pr);
  pi = sum8(pi);
  if (gl == 0) {
    const double2 w = cmul(t, make_double2(pr, pi));
    ww[r] = w;
    const double2 v = vv[r];
    dr_acc += w.x * v.x + w.y * v.y;
    di_acc += w.x * v.y - w.y * v.x;
  }
}

template <bool IN_LDS>
__global__ __launch_bounds__(EIG_THREADS) void k_tridiag(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.x);
  extern __shared__ double smem[];
  __shared__ TriShared sh;
  const int s = a.s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nthr = blockDim.x;
  double2* P = reinterpret_cast<double2*>(smem);
  double2* vv = IN_LDS ? P + tri(s) : P;
  double2* ww = vv + s;
  double2* A = a.G;
  EigWork W = eig_layout(a.work, s, a.kmax);
  if (a.tstamp && tid == 0) a.tstamp[0] = wall_clock64();
  if (IN_LDS) {
    for (int idx = tid; idx < tri(s); idx += nthr) {
      int r = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (tri(r + 1) <= idx) ++r;
      while (tri(r) > idx) --r;
      const int c = idx - tri(r);
      P[idx] = A[(size_t)r * s + c];
    }
  }
  __syncthreads();
  const int grp = tid / RG, gl = tid % RG, ngrp = nthr / RG;
  long long tA = 0, tB = 0, tD = 0, t0 = 0;
  const bool stamp = a.tstamp && tid == 0;
  for (int j = 0; j < s - 1; ++j) {
    const int nj = s - j - 1;
    if (stamp) t0 = wall_clock64();
    if (wave == 0) {
      const double2 alpha = IN_LDS ? P[tri(j + 1) + j] : A[(size_t)(j + 1) * s + j];
      double xn2 = 0.0;
      for (int i = j + 2 + lane; i < s; i += 64) {
        const double2 x = IN_LDS ? P[tri(i) + j] : A[(size_t)i * s + j];
        xn2 += x.x * x.x + x.y * x.y;
      }
      xn2 = wave_sum(xn2);
      const double ajj = IN_LDS ? P[tri(j) + j].x : A[(size_t)j * s + j].x;
      const double2 scal = householder(alpha, xn2, j, ajj, sh, W, lane);
      if (lane == 0) {
        vv[0] = make_double2(1.0, 0.0);
        W.V[(size_t)j * s + j + 1] = make_double2(1.0, 0.0);
      }
      for (int i = 1 + lane; i < nj; i += 64) {
        const double2 x = IN_LDS ? P[tri(j + 1 + i) + j] : A[(size_t)(j + 1 + i) * s + j];
        const double2 v = cmul(x, scal);
        vv[i] = v;
        W.V[(size_t)j * s + j + 1 + i] = v;
      }
    }
    __syncthreads();
    if (stamp) { const long long t1 = wall_clock64(); tA += t1 - t0; t0 = t1; }
    const double2 t = sh.tau;
    if (t.x == 0.0 && t.y == 0.0) continue;
    double dr_acc = 0.0, di_acc = 0.0;
    for (int r = grp; r < nj; r += ngrp) {
      const int R = j + 1 + r;
      if (IN_LDS) {
        matvec_row(r, nj, gl, vv, t, [&](int rr, int c) {
          const int C = j + 1 + c;
          return (c <= rr) ? P[tri(R) + C] : cconj(P[tri(C) + R]);
        }, ww, dr_acc, di_acc);
      } else {
        const double2* row = A + (size_t)R * s + (j + 1);
        matvec_row(r, nj, gl, vv, t, [&](int, int c) { return row[c]; }, ww, dr_acc, di_acc);
      }
    }
    dr_acc = wave_sum(dr_acc);
    di_acc = wave_sum(di_acc);
    if (lane == 0) sh.part[wave] = make_double2(dr_acc, di_acc);
    __syncthreads();
    if (stamp) { const long long t1 = wall_clock64(); tB += t1 - t0; t0 = t1; }
    double dsum_r = 0.0, dsum_i = 0.0;
    for (int w = 0; w < (nthr >> 6); ++w) {
      dsum_r += sh.part[w].x;
      dsum_i += sh.part[w].y;
    }
    const double2 q = cmul(t, make_double2(dsum_r, dsum_i));
    const double2 a2 = make_double2(-0.5 * q.x, -0.5 * q.y);
    // A_sub -= v w'^H + w' v^H with w' = w + a2 v (lower triangle in LDS, full rows in global)
    for (int r = grp; r < nj; r += ngrp) {
      const int R = j + 1 + r;
      const double2 vr = vv[r];
      const double2 wr = make_double2(ww[r].x + a2.x * vr.x - a2.y * vr.y,
                                      ww[r].y + a2.x * vr.y + a2.y * vr.x);
      const int cend = IN_LDS ? r : nj - 1;
      double2* rowp = IN_LDS ? P + tri(R) + (j + 1) : A + (size_t)R * s + (j + 1);
      for (int c = gl; c <= cend; c += RG) {
        const double2 vc = vv[c];
        const double2 wc = make_double2(ww[c].x + a2.x * vc.x - a2.y * vc.y,
                                        ww[c].y + a2.x * vc.y + a2.y * vc.x);
        double2 x = rowp[c];
        x.x -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
        x.y -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
        rowp[c] = x;
      }
    }
    __syncthreads();
    if (stamp) tD += wall_clock64() - t0;
  }
  if (stamp) {
    a.tstamp[4] = tA;
    a.tstamp[5] = tB;
    a.tstamp[6] = tD;
  }
  // last diagonal entry and the Gershgorin interval of T (used by the two later kernels)
  if (tid == 0) W.d[s - 1] = IN_LDS ? P[tri(s - 1) + s - 1].x : A[(size_t)(s - 1) * s + (s - 1)].x;
  __syncthreads();
  if (wave == 0) {
    double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
    for (int i = lane; i < s; i += 64) {
      const double el = i > 0 ? fabs(W.e[i - 1]) : 0.0;
      const double er = i < s - 1 ? fabs(W.e[i]) : 0.0;
      lo = fmin(lo, W.d[i] - el - er);
      hi = fmax(hi, W.d[i] + el + er);
      emax = fmax(emax, er * er);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    emax = wave_max(emax);
    if (lane == 0) {
      const double tn = fmax(fabs(lo), fabs(hi));
      const double pad = 2.0 * DBL_EPSILON * tn * s + DBL_MIN;
      W.bounds[0] = lo - pad;
      W.bounds[1] = hi + pad;
      W.bounds[2] = tn;
      W.bounds[3] = DBL_MIN * fmax(1.0, emax);
      if (a.tstamp) a.tstamp[1] = wall_clock64();
    }
  }
}

// ---- eigenvalues: one wave per eigenvalue -------------------------------------------------------
static constexpr int EV_WAVES = 4;

__global__ __launch_bounds__(64 * EV_WAVES) void k_eigvals(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  extern __shared__ double smem[];
  const int s = a.s, kmax = a.kmax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* dd = smem;
  double* ee2 = dd + s;
  EigWork W = eig_layout(a.work, s, kmax);
  for (int i = tid; i < s; i += blockDim.x) {
    dd[i] = W.d[i];
    ee2[i] = i < s - 1 ? W.e[i] * W.e[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.x * EV_WAVES + wave;
  if (t >= kmax) return;
  const double pivmin = W.bounds[3];
  const double target = 2.0 * DBL_EPSILON * W.bounds[2] + 4.0 * pivmin;
  const int jidx = s - 1 - t;   // ascending index of the t-th largest eigenvalue
  double lo = W.bounds[0], hi = W.bounds[1];
  for (int rd = 0; rd < 40 && hi - lo > target; ++rd) {
    const double x = lo + (hi - lo) * double(lane + 1) / 65.0;
    const int c = sturm_count(dd, ee2, s, x, pivmin);
    const int b = __popcll(__ballot(c <= jidx));
    const double xlo = lo + (hi - lo) * double(b) / 65.0;
    const double xhi = lo + (hi - lo) * double(b + 1) / 65.0;
    lo = xlo;
    hi = xhi;
  }
  if (lane == 0) a.lam[t] = 0.5 * (lo + hi);
  if (a.tstamp && lane == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 2), (unsigned long long)wall_clock64());
}

// ---- eigenvectors of T and back-transformation: one wave per eigenpair ---------------------------
// Twisted factorisation for an isolated eigenvalue x; y gets the unit eigenvector. Single lane.
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
// Single lane; vectors to Y[u*s ..].
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

// u = Q y for one column (wave-cooperative), y real in `yin`, result to U[:, t] (or zero).
__device__ void back_transform_col(const EigArgs& a, const EigWork& W, int s, int kmax, int t,
                                   bool kept, const double* yin, double2* u) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < s; i += 64) u[i] = make_double2(yin[i], 0.0);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  for (int j = s - 2; j >= 0; --j) {
    const double2 tj = W.tau[j];
    if (tj.x == 0.0 && tj.y == 0.0) continue;
    const double2* vj = W.V + (size_t)j * s;
    double dr = 0.0, di = 0.0;
    for (int i = j + 1 + lane; i < s; i += 64) {
      const double2 v = vj[i];
      const double2 x = u[i];
      dr += v.x * x.x + v.y * x.y;
      di += v.x * x.y - v.y * x.x;
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double2 f = cmul(tj, make_double2(dr, di));
    for (int i = j + 1 + lane; i < s; i += 64) {
      const double2 v = vj[i];
      double2 x = u[i];
      x.x -= v.x * f.x - v.y * f.y;
      x.y -= v.x * f.y + v.y * f.x;
      u[i] = x;
    }
  }
  for (int i = lane; i < s; i += 64)
    a.U[(size_t)i * kmax + t] = kept ? u[i] : make_double2(0.0, 0.0);
}

// Register-resident variant for s <= 64 R: lane l holds rows l + 64 q; the next reflector and its tau
// are loaded while the current one is reduced.
template <int R>
__device__ void back_transform_reg(const EigArgs& a, const EigWork& W, int s, int kmax, int t,
                                   bool kept, const double* yin) {
  const int lane = threadIdx.x & 63;
  double2 ur[R], vn[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = lane + 64 * q;
    ur[q] = make_double2(i < s ? yin[i] : 0.0, 0.0);
  }
  int j = s - 2;
  double2 taun = j >= 0 ? W.tau[j] : make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = lane + 64 * q;
    vn[q] = (j >= 0 && i > j && i < s) ? W.V[(size_t)j * s + i] : make_double2(0.0, 0.0);
  }
  for (; j >= 0; --j) {
    double2 vc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) vc[q] = vn[q];
    const double2 tc = taun;
    if (j > 0) {
      taun = W.tau[j - 1];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = lane + 64 * q;
        vn[q] = (i > j - 1 && i < s) ? W.V[(size_t)(j - 1) * s + i] : make_double2(0.0, 0.0);
      }
    }
    if (tc.x == 0.0 && tc.y == 0.0) continue;
    double dr = 0.0, di = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      dr += vc[q].x * ur[q].x + vc[q].y * ur[q].y;
      di += vc[q].x * ur[q].y - vc[q].y * ur[q].x;
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double2 f = cmul(tc, make_double2(dr, di));
#pragma unroll
    for (int q = 0; q < R; ++q) {
      ur[q].x -= vc[q].x * f.x - vc[q].y * f.y;
      ur[q].y -= vc[q].x * f.y + vc[q].y * f.x;
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = lane + 64 * q;
    if (i < s) a.U[(size_t)i * kmax + t] = kept ? ur[q] : make_double2(0.0, 0.0);
  }
}

__device__ void back_transform_any(const EigArgs& a, const EigWork& W, int s, int kmax, int t,
                                   bool kept, const double* yin, double2* u) {
  if (s <= 64) back_transform_reg<1>(a, W, s, kmax, t, kept, yin);
  else if (s <= 128) back_transform_reg<2>(a, W, s, kmax, t, kept, yin);
  else if (s <= 256) back_transform_reg<4>(a, W, s, kmax, t, kept, yin);
  else back_transform_col(a, W, s, kmax, t, kept, yin, u);
}

__global__ __launch_bounds__(256) void k_eigvecs(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  extern __shared__ double smem[];
  const int s = a.s, kmax = a.kmax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  double* dd = smem;
  double* el = dd + s;
  double* region = el + s + 4 * (size_t)s * wave;   // per wave: lp | dp (y later) | um | y
  EigWork W = eig_layout(a.work, s, kmax);
  for (int i = tid; i < s; i += blockDim.x) {
    dd[i] = W.d[i];
    el[i] = i < s - 1 ? W.e[i] : 0.0;
  }
  __syncthreads();
  const int t = blockIdx.x * nw + wave;
  if (t >= kmax) return;
  const double tnorm = W.bounds[2], pivmin = W.bounds[3];
  const double* lam = a.lam;
  // rank selection: keep lam_t > tol^2 lam_0 (descending order), always the first
  int keep = kmax;
  if (a.tol > 0.0) {
    const double cut = a.tol * a.tol * lam[0];
    int c = 0;
    for (int u = lane; u < kmax; u += 64) c += lam[u] > cut;
    c = (int)wave_sum((double)c);
    keep = c < 1 ? 1 : c;
  }
  if (t == 0 && lane == 0) {
    a.kkeep[0] = keep;
    a.inv_sqrt_l0[0] = lam[0] > 0.0 ? 1.0 / sqrt(lam[0]) : 1.0;
  }
  // clusters of non-negligible eigenvalues closer than 1e-3 ||T||; negligible ones (at the rounding
  // level of ||T||) carry no weight and are computed one by one
  const double ortol = 1e-3 * tnorm, tiny = 64.0 * DBL_EPSILON * tnorm;
  auto starts = [&](int u) {
    return u == 0 || u == kmax || lam[u - 1] - lam[u] > ortol || lam[u] <= tiny;
  };
  if (!starts(t)) {   // computed by the wave of the cluster's first member
    if (a.tstamp && lane == 0)
      atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 3), (unsigned long long)wall_clock64());
    return;
  }
  int ce = t + 1;
  while (ce < kmax && !starts(ce)) ++ce;
  double* lp = region;
  double* dp = region + s;
  double* um = region + 2 * s;
  double* y = region + 3 * s;
  double2* u = reinterpret_cast<double2*>(region);   // reuses lp|dp after the twisted solve
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  if (ce == t + 1) {
    if (lane == 0) twisted_vector(dd, el, s, lam[t], pivmin, y, lp, dp, um);
    wave_sync();
    back_transform_any(a, W, s, kmax, t, t < keep, y, u);
  } else {
    // a cluster: if its members are distinct at the rounding level, twisted vectors are accurate up
    // to mixing inside the cluster, so modified Gram-Schmidt over the members gives an orthonormal
    // basis of the cluster's invariant subspace; near-exact degeneracies use inverse iteration.
    double mingap = DBL_MAX;
    for (int m = t + 1; m < ce; ++m) mingap = fmin(mingap, lam[m - 1] - lam[m]);
    if (mingap > 1e-12 * tnorm) {
      double* Yc = W.Y;
      for (int m = t; m < ce; ++m) {
        double* ym = Yc + (size_t)m * s;
        if (lane == 0) twisted_vector(dd, el, s, lam[m], pivmin, y, lp, dp, um);
        wave_sync();
        for (int pass = 0; pass < 2; ++pass) {
          for (int q = t; q < m; ++q) {
            const double* yq = Yc + (size_t)q * s;
            double dot = 0.0;
            for (int i = lane; i < s; i += 64) dot += yq[i] * y[i];
            dot = wave_sum(dot);
            for (int i = lane; i < s; i += 64) y[i] -= dot * yq[i];
            wave_sync();
          }
        }
        double nrm = 0.0;
        for (int i = lane; i < s; i += 64) nrm += y[i] * y[i];
        nrm = wave_sum(nrm);
        const double inv = 1.0 / sqrt(nrm);
        for (int i = lane; i < s; i += 64) ym[i] = y[i] * inv;
        __threadfence_block();
        wave_sync();
      }
    } else if (lane == 0) {
      cluster_vectors(dd, el, s, lam, t, ce, tnorm, W.Y, W.lu + (size_t)t * 5 * s);
    }
    wave_sync();
    for (int m = t; m < ce; ++m) {
      back_transform_any(a, W, s, kmax, m, m < keep, W.Y + (size_t)m * s, u);
      wave_sync();
    }
  }
  if (a.tstamp && lane == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 3), (unsigned long long)wall_clock64());
  if (a.tstamp && lane == 0 && ce > t + 1) atomicAdd(reinterpret_cast<unsigned long long*>(a.tstamp + 7), 1ull);
}

size_t eig_lds_bytes(int s, int kmax, bool in_lds) {
  (void)kmax;
  return (in_lds ? (size_t)16 * (s * (size_t)(s + 1) / 2) : 0) + (size_t)s * (2 * 16) + 64;
}

hipError_t launch_eig(const EigArgs& a, hipStream_t st) {
  if (a.s <= 0 || a.kmax <= 0 || a.kmax > a.s || a.batch <= 0) return hipErrorInvalidValue;
  const bool in_lds = a.s <= EIG_LDS_MAX;
  const size_t lds = eig_lds_bytes(a.s, a.kmax, in_lds);
  if (lds > 160 * 1024 - 512) return hipErrorInvalidValue;
  if (in_lds) {
    (void)hipFuncSetAttribute((const void*)k_tridiag<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_tridiag<true>, dim3(a.batch), dim3(EIG_THREADS), lds, st, a);
  } else {
    (void)hipFuncSetAttribute((const void*)k_tridiag<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_tridiag<false>, dim3(a.batch), dim3(EIG_THREADS), lds, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds2 = (size_t)16 * a.s;
  hipLaunchKernelGGL(k_eigvals, dim3((a.kmax + EV_WAVES - 1) / EV_WAVES, a.batch),
                     dim3(64 * EV_WAVES), lds2, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nw = a.s <= 1000 ? 4 : (a.s <= 1900 ? 2 : 1);
  const size_t lds3 = (size_t)a.s * (2 * 8 + (size_t)nw * 4 * 8) + 64;
  if (lds3 > 160 * 1024 - 512) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)k_eigvecs, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds3);
  hipLaunchKernelGGL(k_eigvecs, dim3((a.kmax + nw - 1) / nw, a.batch), dim3(64 * nw), lds3, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
__global__ void k_form_l_nside(const double2* V, const double* lam, const int* kkeep, int n,
                               int kmax, void* L, int tl, int64_t bs) {
  const int b = blockIdx.y;
  V = inst_ptr(V, bs, b);
  lam = inst_ptr(lam, bs, b);
  kkeep = inst_ptr(kkeep, bs, b);
  L = inst_ptr(L, bs, b);
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
                               int kmax, void* L, DType tl, int batch, int64_t bs, hipStream_t st) {
  const int64_t tot = (int64_t)kmax * n;
  if (tot == 0 || batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_form_l_nside, dim3((unsigned)((tot + 255) / 256), batch), dim3(256), 0, st,
                     V, lam, kkeep, n, kmax, L, (int)tl, bs);
  return hipGetLastError();
}

}  // namespace cbc
