// Device helpers and the scratch layout shared by the eigensolver's translation units (the
// one-stage reduction and tridiagonal eigenpairs in eig.hip, the two-stage band reduction and its
// back-transformation in eig_band.hip).
#pragma once
#include <float.h>

#include "cbc_internal.h"
#include "device_status.h"

namespace cbc {

static constexpr int EIG_THREADS = 1024;
static constexpr int EIG_LDS_MAX = 128;   // largest s whose packed triangle stays in LDS
static constexpr int RG = 8;              // lanes per row group in the matrix-vector product
static constexpr int TRI_U = 4;           // elements per lane whose LDS loads are issued together

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
// a / b through the hardware reciprocal refined by one Newton step (relative error about the square
// of the hardware estimate's; used only in the Sturm counts and the twisted factorisation, which
// tolerate relative errors far above one ulp per step and whose callers guard b away from zero).
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}

// Layout of the scratch buffer (doubles).
static constexpr int MW_MAX_WG = 256;     // workgroups of the multi-workgroup reduction, at most
struct EigWork {
  double* d;      // s
  double* e;      // s
  double2* tau;   // s
  double* bounds; // 8: lo, hi, tnorm, pivmin, the (kmax+1)-th largest eigenvalue
  double2* V;     // s * s   reflector j at V[j*s + i], i > j, V[j*s+j+1] = 1
  double* Y;      // kmax * s   cluster eigenvectors of T at Y[t*s + i]
  double* lu;     // kmax * 5 * s
  // multi-workgroup reduction only (each double-buffered by the parity of the column)
  double2* ybuf;  // 2 * s       products A v of the current column
  double2* prow;  // 2 * s       next pivot row, published by its owner
  // blocked back-transformation: the triangular factor of each block of BT_NB reflectors
  double2* tfac;  // bt_blocks(s) * BT_NB * BT_NB
  unsigned* sync; // MW_MAX_WG + 16 words: barrier flags or arrival counters, then a time-out flag
};
static constexpr int BT_NB = 32;   // reflectors per block of the blocked back-transformation
__host__ __device__ inline int bt_blocks(int s) { return s > 1 ? (s - 1 + BT_NB - 1) / BT_NB : 0; }
__host__ __device__ inline EigWork eig_layout(double* w, int s, int kmax) {
  EigWork L;
  L.d = w;
  L.e = w + s;
  L.tau = reinterpret_cast<double2*>(w + 2 * (size_t)s);
  L.bounds = w + 4 * (size_t)s;
  L.V = reinterpret_cast<double2*>(w + 4 * (size_t)s + 8);
  L.Y = w + 4 * (size_t)s + 8 + 2 * (size_t)s * s;
  L.lu = L.Y + (size_t)kmax * s;
  L.ybuf = reinterpret_cast<double2*>(L.lu + 5 * (size_t)kmax * s);
  L.prow = L.ybuf + 2 * (size_t)s;
  L.tfac = L.prow + 2 * (size_t)s;
  L.sync = reinterpret_cast<unsigned*>(L.tfac + (size_t)bt_blocks(s) * BT_NB * BT_NB);
  return L;
}
static constexpr int MW_SYNC_BYTES = 4 * (MW_MAX_WG + 16);
// doubles of the layout above (the two-stage reduction's scratch follows it)
__host__ __device__ inline size_t eig_base_doubles(int s, int kmax) {
  return 4 * (size_t)s + 8 + 2 * (size_t)s * s + (size_t)kmax * s + 5 * (size_t)kmax * s +
         4 * (size_t)s + 4 * (size_t)s + 2 * (size_t)bt_blocks(s) * BT_NB * BT_NB +
         MW_SYNC_BYTES / 8 + 64;
}
// two-stage reduction (eig_band.hip): scratch beyond eig_base_doubles, the reduction of G to T
// (d, e and the Gershgorin bounds in the common layout) and the back-transformation into U
size_t band_work_doubles(int s);
hipError_t launch_band_reduction(const EigArgs& a, hipStream_t st);
hipError_t launch_bt_band(const EigArgs& a, hipStream_t st);
// EigArgs of instance b (every pointer except the time stamps advances by a.bs bytes)
__device__ inline EigArgs eig_inst(const EigArgs& a0, int b) {
  EigArgs a = a0;
  a.G = inst_ptr(a0.G, a0.bs, b);
  a.U = inst_ptr(a0.U, a0.bs, b);
  a.lam = inst_ptr(a0.lam, a0.bs, b);
  a.kkeep = inst_ptr(a0.kkeep, a0.bs, b);
  a.inv_sqrt_l0 = inst_ptr(a0.inv_sqrt_l0, a0.bs, b);
  a.work = inst_ptr(a0.work, a0.bs, b);
  a.status = inst_ptr(a0.status, a0.bs, b);
  a.rec = inst_ptr(a0.rec, a0.bs, b);
  return a;
}

// a double from lane `l` (wave-uniform) of the wave
__device__ __forceinline__ double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ double2 readlane_z(double2 v, int l) {
  return make_double2(readlane_d(v.x, l), readlane_d(v.y, l));
}
// Gershgorin interval of T and the pivot floor of the Sturm counts; one wave. A non-finite T (a
// Gram with NaN or infinite entries) raises CBC_ENOTPD.
__device__ inline void tri_bounds(EigWork& W, int s, long long* tstamp, int* status) {
  const int lane = threadIdx.x & 63;
  {
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
      if (!isfinite(lo) || !isfinite(hi)) raise_status(status, CBC_ENOTPD);
      const double tn = fmax(fabs(lo), fabs(hi));
      const double pad = 2.0 * DBL_EPSILON * tn * s + DBL_MIN;
      W.bounds[0] = lo - pad;
      W.bounds[1] = hi + pad;
      W.bounds[2] = tn;
      W.bounds[3] = DBL_MIN * fmax(1.0, emax);
      if (tstamp) tstamp[1] = wall_clock64();
    }
  }
}

// ---- XCD-aware launches ------------------------------------------------------------------------
// The kernels after the reduction read what it wrote for an instance (T, the reflectors, Y). For
// small Grams and few instances their grids are launched a.spread = 8 times wider along x and only
// the work-groups whose linear index is congruent to the instance modulo 8 work: work-groups are
// placed on the 8 XCDs round-robin by linear index, so an instance's work stays on one XCD and its
// reflectors are fetched into one L2 (measured at s = 128: 2.9 -> 0.9 MB of HBM traffic per solve;
// the single-workgroup reduction of instance b runs on XCD b mod 8 as well). Large Grams, whose
// back-transformation needs more than one XCD's compute units, and batches of 8 or more instances,
// which spread over the XCDs anyway, use plain grids (spread = 1).
static constexpr int XCD_SPREAD = 8;
__device__ __forceinline__ bool xcd_own(int spread) {
  return (int)(blockIdx.x % spread) == (int)(blockIdx.y % spread);
}

}  // namespace cbc
