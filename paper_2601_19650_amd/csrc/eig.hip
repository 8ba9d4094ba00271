// FP64 Hermitian eigensolver for the truncation step.
//
// The compression keeps the top-k singular subspace of the joined-leg matrix (Sec. III A leaves the
// compression method open and names the singular value decomposition). On the GPU it is reached through the
// FP64 Gram matrix G of that matrix: its top-k eigenvectors span the same subspace and its
// eigenvalues are the squared singular values.
//
// One G is solved by a reduction to a real symmetric tridiagonal T = Q^H G Q (reflectors
// H_j = I - tau_j v_j v_j^H, real sub-diagonal), then the top-kmax eigenpairs of T, then the
// back-transformation u = Q y:
//   1. reduction: for s <= EIG_LDS_MAX one workgroup (k_tridiag) holds the packed lower triangle in
//      LDS; the Hermitian matrix-vector product uses groups of 8 lanes per row and DPP reductions,
//      w^H v and w' are formed once by wave 0 (sums in a fixed order: bitwise reproducible); while
//      15 waves apply the rank-2 update (again 8 lanes per row), wave 0 updates the next column
//      itself and forms its reflector (look-ahead), so a column costs two workgroup barriers.
//      Larger s use k_tridiag_mw: the rows are spread over many workgroups (held in registers)
//      and every column costs one grid-wide barrier; its last 128 columns are left to k_tridiag.
//   2. k_eigvals, one wave per eigenvalue over many workgroups: multisection on Sturm counts (64
//      points of the current interval per round).
//   3. eigenvectors of T by a twisted factorisation T - lambda I = N_r Delta N_r^T, one wave per
//      eigenpair; eigenvalues closer than 1e-3 ||T|| form clusters that are re-orthogonalised (or,
//      for near-exact degeneracies, computed by inverse iteration); then the back-transformation:
//      for s <= 256 one wave per eigenpair applying the reflectors streamed from L2, above that in
//      blocks of 32 reflectors (compact WY: the factors formed alongside the eigenvalues, then
//      k_bt_wy).
#include <float.h>

#include <mutex>

#include "eig_common.h"

namespace cbc {

size_t eig_work_doubles(int s, int kmax) {
  return eig_base_doubles(s, kmax) + (s > EIG_LDS_MAX ? band_work_doubles(s) : 0);
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
  double2 tau[2];   // tau of the current and of the next column (by parity)
  double2 zero;     // read in place of w past the trailing size
};

// w' = w + a2 v, the corrected product of one row
__device__ __forceinline__ double2 wprime(double2 w, double2 v, double2 a2) {
  return make_double2(w.x + a2.x * v.x - a2.y * v.y, w.y + a2.x * v.y + a2.y * v.x);
}
// x - (v_r w'_c^* + w'_r v_c^*): one element of the rank-2 update, as a chain of FMAs
__device__ __forceinline__ double2 rank2(double2 x, double2 vr, double2 wr, double2 vc, double2 wc) {
  x.x = fma(-vr.x, wc.x, x.x);
  x.x = fma(-vr.y, wc.y, x.x);
  x.x = fma(-wr.x, vc.x, x.x);
  x.x = fma(-wr.y, vc.y, x.x);
  x.y = fma(-vr.y, wc.x, x.y);
  x.y = fma(vr.x, wc.y, x.y);
  x.y = fma(-wr.y, vc.x, x.y);
  x.y = fma(wr.x, vc.y, x.y);
  return x;
}

// Householder reflector of column C from x = A[C+1.., C] (alpha = x[0], xn2 = |x[1..]|^2); lane 0
// records tau, beta and the diagonal a_CC. Returns the scaling 1/(alpha - beta) that maps x[1..] to
// the reflector.
__device__ inline double2 householder(double2 alpha, double xn2, int C, double a_cc, double2& tau,
                                      EigWork& W, int lane) {
  double2 t = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
  double beta = alpha.x;
  if (!(xn2 == 0.0 && alpha.y == 0.0)) {
    // |x| and 1/|x| from the hardware reciprocal square root refined by two Newton steps, 1/|alpha -
    // beta|^2 from the hardware reciprocal refined likewise (each step squares the relative error,
    // so two leave about one ulp whatever the estimate's accuracy; the column norm is positive here)
    const double n2 = alpha.x * alpha.x + alpha.y * alpha.y + xn2;
    double rn = __builtin_amdgcn_rsq(n2);
    rn = fma(0.5 * rn, fma(-n2 * rn, rn, 1.0), rn);
    rn = fma(0.5 * rn, fma(-n2 * rn, rn, 1.0), rn);
    const double nrm = n2 * rn;
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    const double rb = alpha.x >= 0.0 ? -rn : rn;   // 1 / beta
    const double ar = alpha.x - beta, ai = alpha.y;
    const double den = ar * ar + ai * ai;
    double rden = __builtin_amdgcn_rcp(den);
    rden = fma(rden, fma(-den, rden, 1.0), rden);
    rden = fma(rden, fma(-den, rden, 1.0), rden);
    t = make_double2(-ar * rb, -ai * rb);
    scal = make_double2(ar * rden, -ai * rden);
  }
  if (lane == 0) {
    tau = t;
    W.tau[C] = t;
    W.e[C] = beta;
    W.d[C] = a_cc;
  }
  return scal;
}

// Reflector of the next column, by one wave (look-ahead). xin holds column C = j + 1 of the
// trailing matrix as it was before the rank-2 update of column j (row C + r in lane r mod 64, rows
// past the end repeat the last one); with upd the update is applied here (v and w' of row C + r in
// vr, wr, the same lanes), while the other waves update every other column of the trailing matrix.
// Records d[C] and, below the last column, the reflector of column C into vnext, tau and the
// workspace.
__device__ inline void next_reflector(const double2 xin[2], int s, int j, bool upd,
                                      const double2 vr[2], const double2 wr[2], double2* vnext,
                                      double2& tau, EigWork& W, int ldv, int lane) {
  const int C = j + 1, n = s - C;
  double2 x[2] = {xin[0], xin[1]};
  if (upd) {
    const double2 v0 = readlane_z(vr[0], 0), w0 = readlane_z(wr[0], 0);
#pragma unroll
    for (int k = 0; k < 2; ++k) x[k] = rank2(x[k], vr[k], wr[k], v0, w0);
  }
  const double acc = readlane_d(x[0].x, 0);
  if (C == s - 1) {
    if (lane == 0) W.d[C] = acc;
    return;
  }
  const double2 alpha = readlane_z(x[0], 1);
  double xn2 = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = lane + 64 * k;
    if (r >= 2 && r < n) xn2 += x[k].x * x[k].x + x[k].y * x[k].y;
  }
  xn2 = wave_sum(xn2);
  const double2 scal = householder(alpha, xn2, C, acc, tau, W, lane);
  if (lane == 0) {
    vnext[0] = make_double2(1.0, 0.0);
    W.V[(size_t)C * ldv + C + 1] = make_double2(1.0, 0.0);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = lane + 64 * k;
    if (r >= 2 && r < n) {
      const double2 v = cmul(x[k], scal);
      vnext[r - 1] = v;
      W.V[(size_t)C * ldv + C + r] = v;
    }
  }
}

// column C of the packed triangle, rows C + r in lane r mod 64 (rows past s - 1 repeat the last)
__device__ __forceinline__ void load_column(const double2* P, int s, int C, int lane, double2 x[2]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) x[k] = P[tri(C + min(lane + 64 * k, s - 1 - C)) + C];
}


// With sfull > a.s the kernel reduces the trailing a.s x a.s block (rows and columns from
// sfull - a.s on, stored densely in G with row stride a.s) that the multi-workgroup reduction of an
// sfull x sfull Gram left after its first sfull - a.s reflectors, and records its reflectors, d and
// e at those offsets of the sfull layout; the Gershgorin interval is then that of the whole T.
__global__ __launch_bounds__(EIG_THREADS) void k_tridiag(EigArgs a0, int sfull) {
  const EigArgs a = eig_inst(a0, blockIdx.x);
  extern __shared__ double smem[];
  __shared__ TriShared sh;
  const int s = a.s;
  // the wave index as a scalar: the update's rows and branches are then uniform per wave
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthr = blockDim.x;
  double2* P = reinterpret_cast<double2*>(smem);
  double2* vb = P + tri(s);     // reflectors of the current and the next column (by parity)
  double2* ww = vb + 2 * s;
  double2* A = a.G;
  const int off = sfull - s, ldv = sfull;
  EigWork Wf = eig_layout(a.work, sfull, a.kmax);
  EigWork W = Wf;
  W.d += off;
  W.e += off;
  W.tau += off;
  W.V += (size_t)off * sfull + off;
  if (a.tstamp && tid == 0 && off == 0) a.tstamp[0] = wall_clock64();
  if (tid == 0) sh.zero = make_double2(0.0, 0.0);
  for (int idx = tid; idx < tri(s); idx += nthr) {
    int r = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while (tri(r + 1) <= idx) ++r;
    while (tri(r) > idx) --r;
    const int c = idx - tri(r);
    P[idx] = A[(size_t)r * s + c];
  }
  __syncthreads();
  if (wave == 0) {
    double2 x0[2];
    load_column(P, s, 0, lane, x0);
    next_reflector(x0, s, -1, false, x0, x0, vb, sh.tau[0], W, ldv, lane);
  }
  __syncthreads();
  const int grp = tid / RG, gl = tid % RG, ngrp = nthr / RG;
  long long tL = 0, tB = 0, tD = 0, t0 = 0;
  const bool stamp = a.tstamp && tid == 0;
  for (int j = 0; j < s - 1; ++j) {
    const int nj = s - j - 1;
    const double2* vv = vb + (j & 1) * s;
    double2* vn = vb + ((j + 1) & 1) * s;
    if (stamp) t0 = wall_clock64();
    const double2 t = sh.tau[j & 1];
    const bool upd = __builtin_amdgcn_readfirstlane(!(t.x == 0.0 && t.y == 0.0));
    // wave 0: column j + 1 (not written again before the look-ahead) and v of its rows, early
    double2 xcol[2], vk[2], wk[2];
    if (wave == 0) {
      load_column(P, s, j + 1, lane, xcol);
#pragma unroll
      for (int k = 0; k < 2; ++k) vk[k] = vv[min(lane + 64 * k, nj - 1)];
    }
    if (upd) {
      // y = A v over the trailing rows, groups of RG lanes per row; w = tau y
      for (int r = grp; r < nj; r += ngrp) {
        const int R = j + 1 + r;
        // row part (stored, contiguous) then column part (conjugated, addressed incrementally:
        // tri(C + RG) = tri(C) + RG C + RG (RG + 1) / 2)
        // (pointer-stepped loops: the fewest integer instructions per element)
        const double2* xp = P + tri(R) + (j + 1) + gl;
        const double2* vp = vv + gl;
        double pr = 0.0, pi = 0.0;
        for (const double2* ve = vv + r; vp <= ve; vp += RG, xp += RG) {
          const double2 x = *xp, v = *vp;
          pr = fma(x.x, v.x, pr);
          pr = fma(-x.y, v.y, pr);
          pi = fma(x.x, v.y, pi);
          pi = fma(x.y, v.x, pi);
        }
        const int c = r + 1 + (((gl - r - 1) % RG) + RG) % RG;
        const int C = j + 1 + c;
        xp = P + tri(C) + R;
        vp = vv + c;
        for (int step = RG * C + RG * (RG + 1) / 2; vp < vv + nj; vp += RG, xp += step, step += RG * RG) {
          const double2 x = *xp, v = *vp;
          pr = fma(x.x, v.x, pr);
          pr = fma(x.y, v.y, pr);
          pi = fma(x.x, v.y, pi);
          pi = fma(-x.y, v.x, pi);
        }
        pr = sum8(pr);
        pi = sum8(pi);
        if (gl == 0) ww[r] = cmul(t, make_double2(pr, pi));
      }
      __syncthreads();
      if (wave == 0) {
        // w' = w + a2 v with a2 = -tau (w^H v) / 2, formed once (kept in wk for the look-ahead)
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int r = lane + 64 * k;
          wk[k] = *(r < nj ? ww + r : &sh.zero);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          dr += wk[k].x * vk[k].x + wk[k].y * vk[k].y;
          di += wk[k].x * vk[k].y - wk[k].y * vk[k].x;
        }
        dr = wave_sum(dr);
        di = wave_sum(di);
        const double2 q = cmul(t, make_double2(dr, di));
        const double2 a2 = make_double2(-0.5 * q.x, -0.5 * q.y);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int r = lane + 64 * k;
          wk[k] = wprime(wk[k], vk[k], a2);
          if (r < nj) ww[r] = wk[k];
        }
      }
      __syncthreads();
    }
    if (stamp) { const long long t1 = wall_clock64(); tB += t1 - t0; t0 = t1; }
    if (wave == 0) {
      next_reflector(xcol, s, j, upd, vk, wk, vn, sh.tau[(j + 1) & 1], W, ldv, lane);
      if (stamp) tL += wall_clock64() - t0;
    } else if (upd) {
      // A -= v w'^H + w' v^H on rows r >= 1 and columns 1 <= c <= r of the trailing matrix (column 0
      // belongs to the look-ahead): groups of RG lanes per row, rows dealt to the groups of waves
      // 1.., TRI_U elements per lane loaded together, then updated and stored; an element past the
      // row end repeats element c0 and stores the same value to it
      const int nug = ngrp - 64 / RG;   // row groups outside wave 0
      for (int r = 1 + grp - 64 / RG; r < nj; r += nug) {
        const int R = j + 1 + r;
        const double2 vr = vv[r];
        const double2 wr = ww[r];
        double2* rowp = P + tri(R) + (j + 1);
        for (int c0 = 1 + gl; c0 <= r; c0 += TRI_U * RG) {
          int cc[TRI_U];
          double2 vc[TRI_U], wc[TRI_U], x[TRI_U];
#pragma unroll
          for (int u = 0; u < TRI_U; ++u) {
            const int c = c0 + u * RG;
            cc[u] = c <= r ? c : c0;
            vc[u] = vv[cc[u]];
            wc[u] = ww[cc[u]];
            x[u] = rowp[cc[u]];
          }
#pragma unroll
          for (int u = 0; u < TRI_U; ++u) x[u] = rank2(x[u], vr, wr, vc[u], wc[u]);
#pragma unroll
          for (int u = 0; u < TRI_U; ++u) rowp[cc[u]] = x[u];
        }
      }
    }
    __syncthreads();
    if (stamp) tD += wall_clock64() - t0;
  }
  if (stamp && off == 0) {
    a.tstamp[4] = tL;
    a.tstamp[5] = tB;
    a.tstamp[6] = tD;
  }
  // the Gershgorin interval of T (used by the two later kernels)
  if (wave == 0) tri_bounds(Wf, sfull, a.tstamp, a.status);
}

// ---- multi-workgroup Householder reduction (s > EIG_LDS_MAX) ------------------------------------
// The rows of G are dealt cyclically to nwg workgroups (row r to workgroup r mod nwg) and stay in
// their threads' registers for the whole reduction. Thread t of every workgroup owns the columns t,
// t + 512, ...: its entries of the owned rows, of the reflector v_j, of w_j and of the next
// reflector live in its registers, so that a column moves no row data through LDS. Column j costs
// one grid-wide barrier:
//   (1) barrier: each workgroup adds its arrival to one of eight counters and waits until all
//       eight have counted every workgroup of their group;
//   (2) every workgroup fetches all of y = A v_j (published by the rows' owners) and the row j+1
//       its owner published one column earlier, and forms w_j = tau y - |tau|^2/2 (v_j^H y)^* v_j;
//   (3) it builds row j+1 of the updated matrix (A -= v_j w_j^H + w_j v_j^H) and from it the next
//       reflector v_{j+1}, identically in every workgroup;
//   (4) one pass over its rows applies the rank-2 update and accumulates the products
//       y' = A' v_{j+1} of the next column (reduced over groups of eight lanes, then from LDS); the
//       owner of row j+2 publishes that row.
// Reductions are summed in a fixed order, so every workgroup holds bitwise the same v and w.
// The barrier waits are bounded: after timeout_ticks of the 100 MHz wall clock (2 s) a workgroup
// raises a flag, every workgroup leaves at its next barrier, d[0] is set to NaN and the call's
// status word receives CBC_ETIMEOUT.
static constexpr int MW_THREADS = 512;
static constexpr int MW_WAVES = MW_THREADS / 64;
static constexpr int MW_EPT = 3;                    // columns per thread, at most: s <= 1536
static constexpr int MW_ROWS_MAX = 16;              // rows per workgroup, at most (row slots in LDS)
// The rows a workgroup owns live in its threads' registers, EPT entries of each row per thread. The
// cap on a workgroup's row bytes below keeps that share at 21 complex entries per thread at most.
static constexpr size_t MW_ROW_BUDGET = 152 * 1024;
// rows per workgroup of the instantiated kernels, at most, by columns per thread
__host__ __device__ constexpr int mw_rows_max(int ept) {
  return ept == 1 ? 3 : ept == 2 ? 5 : ept == 3 ? 7 : 0;
}

static constexpr int MW_TARGET_WG = 208;            // workgroups aimed at (see mw_shape)
// The last MW_TAIL columns are reduced by the one-workgroup kernel (LDS-resident packed triangle),
// whose column costs less than a grid barrier once the trailing matrix is that small.
static constexpr int MW_TAIL = EIG_LDS_MAX;

struct MwShape {
  int nwg, rows;
};
// Rows per workgroup: as few as keep the workgroup count near MW_TARGET_WG, and no more than the
// row budget. Fewer rows shorten the per-column update and product pass of every workgroup, more
// workgroups lengthen the grid barrier; measured on MI355X at s = 1024 (per column: update,
// barrier): 9 rows / 114 workgroups 4.26 + 2.45 us, 6 / 171 2.94 + 2.65, 5 / 205 2.49 + 2.86,
// 4 / 256 2.04 + 3.70. Per solve, against the former rule (as many rows as fit in LDS, at least
// one workgroup per 16 rows): s = 256 2.45 -> 1.66 ms, 420 4.44 -> 3.2, 700 8.3 -> 5.9, 1024
// 12.0 -> 10.7 (targets of 128 and 256 workgroups were slower above s = 420).
__host__ __device__ inline MwShape mw_shape(int s) {
  int fit = (int)(MW_ROW_BUDGET / (16 * (size_t)s));
  if (fit > MW_ROWS_MAX) fit = MW_ROWS_MAX;
  if (fit < 1) fit = 1;
  int rows = (s + MW_TARGET_WG - 1) / MW_TARGET_WG;
  if (rows > fit) rows = fit;
  MwShape m;
  m.nwg = (s + rows - 1) / rows;
  m.rows = (s + m.nwg - 1) / m.nwg;
  return m;
}
static size_t mw_row_bytes(int s) { return (size_t)mw_shape(s).rows * s * 16; }

// the two-stage path: panels of up to 2048 rows (two per thread of the panel kernel)
static constexpr int EIG_MAX_S = 2048 + 16;
bool eig_size_supported(int s) { return s >= 1 && s <= EIG_MAX_S; }
static bool mw_size_supported(int s) {
  return s > EIG_LDS_MAX && s <= MW_EPT * MW_THREADS && mw_shape(s).nwg <= MW_MAX_WG &&
         mw_row_bytes(s) <= MW_ROW_BUDGET &&
         mw_shape(s).rows <= mw_rows_max((s + MW_THREADS - 1) / MW_THREADS);
}
// The one-stage multi-workgroup reduction is the faster one where it applies (measured on MI355X,
// s = 1024: 6.8 ms against 25.6 ms for the two-stage path, per solve), but its workgroups wait for
// each other: it is used for single instances queued eagerly or in the library's own graphs, whose
// launches the device-wide gate orders; batches and calls recorded into a caller's capture take the
// two-stage path, which has no cross-workgroup waits.
int eig_pick_reduction(int s, int batch, bool caller_capture) {
  return mw_size_supported(s) && batch == 1 && !caller_capture ? 1 : 0;
}
bool eig_needs_gate(int s) { return mw_size_supported(s); }

// ---- device-wide order of the multi-workgroup reductions ------------------------------------------
// Two multi-workgroup reductions running at once on one device could each hold part of the compute
// units while waiting for workgroups of their own that cannot be placed. Every such launch queued
// eagerly (a kernel, or a graph of the library's that holds one) is therefore ordered after the
// previous one on the device through one event per device. Nothing is recorded inside a stream
// capture: a capture of the library's own is launched as a graph, which is ordered as a whole, and
// calls recorded into a caller's capture use the two-stage reduction instead.
namespace {
constexpr int GATE_MAX_DEV = 64;
struct Gate {
  std::mutex mu;
  hipEvent_t ev[GATE_MAX_DEV] = {};
  hipStream_t last[GATE_MAX_DEV] = {};
};
Gate& gate() {
  static Gate g;
  return g;
}
hipError_t gate_state(hipStream_t st, int& dev, bool& cap) {
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= GATE_MAX_DEV) return hipErrorInvalidDevice;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  cap = false;
  if (st != nullptr) {
    e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return e;
    cap = cs != hipStreamCaptureStatusNone;
  }
  return hipSuccess;
}
}  // namespace

hipError_t mw_gate_enter(hipStream_t st) {
  int dev;
  bool cap;
  hipError_t e = gate_state(st, dev, cap);
  if (e != hipSuccess || cap) return e;
  Gate& g = gate();
  std::lock_guard<std::mutex> lk(g.mu);
  if (g.ev[dev] && g.last[dev] != st) e = hipStreamWaitEvent(st, g.ev[dev], 0);
  return e;
}

hipError_t mw_gate_leave(hipStream_t st) {
  int dev;
  bool cap;
  hipError_t e = gate_state(st, dev, cap);
  if (e != hipSuccess || cap) return e;
  Gate& g = gate();
  std::lock_guard<std::mutex> lk(g.mu);
  if (!g.ev[dev]) {
    e = hipEventCreateWithFlags(&g.ev[dev], hipEventDisableTiming);
    if (e != hipSuccess) {
      g.ev[dev] = nullptr;
      return e;
    }
  }
  e = hipEventRecord(g.ev[dev], st);
  if (e != hipSuccess) return e;
  g.last[dev] = st;
  return hipSuccess;
}

// Data exchanged between the workgroups (products, partial sums, pivot rows) is written and read
// with device-coherent atomic accesses, which go to the point of coherence without caching in the
// per-XCD L2. The barrier then only has to order them against the arrival flags (each workgroup
// waits for its own stores to complete before publishing its flag) and needs neither an L2
// write-back nor an L2 invalidation, so the rows, the code and everything else stay cached.
__device__ __forceinline__ void cstore(double2* p, double2 v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 cload(const double2* p) {
  double2 v;
  v.x = __hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// Barrier number `it`; sync[MW_MAX_WG] = time-out flag. Below MW_COUNT_MIN workgroups sync[q] is
// the last barrier workgroup q reached and every workgroup polls all flags. From MW_COUNT_MIN on
// (where that polling traffic grows with the square of the count) workgroup q adds one to the
// arrival counter of its group q mod 8, sync[(q mod 8) * MW_CTR_STRIDE] (eight counters on lines of
// their own, so that the additions spread), and every workgroup polls the eight counters, one per
// lane, until each holds `it` times its group's workgroup count.
static constexpr int MW_COUNT_MIN = 64;
static constexpr int MW_CTR_STRIDE = 32;   // words: one 128-byte line per counter
static_assert(8 * MW_CTR_STRIDE <= MW_MAX_WG, "the counters share the per-workgroup flag words");

__device__ bool mw_sync(unsigned* sync, int nwg, unsigned it, int* ok_sh, long long timeout) {
  // every wave's exchanged-data stores have completed before the workgroup publishes its arrival
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < 64) {
    const bool count = nwg >= MW_COUNT_MIN;
    if (tid == 0) {
      if (count)
        __hip_atomic_fetch_add(&sync[(blockIdx.x & 7) * MW_CTR_STRIDE], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_store(&sync[blockIdx.x], it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    const long long t0 = wall_clock64();
    // arrivals group `tid` must have counted (count mode, lanes 0..7; every group is non-empty)
    const unsigned need = tid < 8 ? it * (unsigned)((nwg - tid + 7) / 8) : 0u;
    for (;;) {
      int done = 1;
      if (count) {
        if (tid < 8)
          done = __hip_atomic_load(&sync[tid * MW_CTR_STRIDE], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) >= need;
      } else {
        for (int q = tid; q < nwg; q += 64)
          done &= __hip_atomic_load(&sync[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= it;
      }
      if (__all(done)) break;
      const int err =
          __hip_atomic_load(&sync[MW_MAX_WG], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
      if (__any(err) || timeout < 0 || wall_clock64() - t0 > timeout) {
        if (tid == 0) __hip_atomic_store(&sync[MW_MAX_WG], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (tid == 0) *ok_sh = ok;
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return *ok_sh != 0;
}

// Block-wide sum of every thread's complex value in a fixed order; `red` holds one slot per wave and
// is read by every thread after the caller's next __syncthreads (sum_red below).
// the same for a real value (the slot's imaginary part is not written)
__device__ __forceinline__ void put_red_re(double re, double2* red) {
  re = wave_sum(re);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6].x = re;
}
// the real part of sum_red
template <int NW_>
__device__ __forceinline__ double sum_red_re(const double2* red) {
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < NW_; ++q) t += red[q].x;
  return t;
}
__device__ __forceinline__ void put_red(double re, double im, double2* red) {
  re = wave_sum(re);
  im = wave_sum(im);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(re, im);
}
__device__ __forceinline__ double2 sum_red(const double2* red) {
  double2 t = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < MW_WAVES; ++q) {
    t.x += red[q].x;
    t.y += red[q].y;
  }
  return t;
}

template <int EPT, int R>   // columns per thread (s <= EPT * MW_THREADS), rows per workgroup at most
__global__ __launch_bounds__(MW_THREADS) void k_tridiag_mw(EigArgs a0, int nwg, int tail) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int wg = blockIdx.x;
  const int s = a.s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nr = wg < s ? (s - wg + nwg - 1) / nwg : 0;   // rows owned: wg, wg + nwg, ...
  __shared__ double2 red_c[MW_WAVES], red_n[MW_WAVES];
  __shared__ double2 racc[R][MW_WAVES * 8];            // row partials of groups of 8 lanes
  __shared__ double2 rv[MW_ROWS_MAX], ry[MW_ROWS_MAX];   // v_j and y at the owned rows' indices
  __shared__ double2 bc[3];                               // y[j+1]; row j+1 at j+1 and j+2
  __shared__ int ok_sh;
  EigWork W = eig_layout(a.work, s, a.kmax);
  const bool writer = wg == 0;
  if (a.tstamp && writer && tid == 0) a.tstamp[0] = wall_clock64();
  // the owned rows, in registers: Ar[q][e] is row wg + q nwg at column tid + e MW_THREADS
  double2 Ar[R][EPT];
#pragma unroll
  for (int q = 0; q < R; ++q) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int c = tid + e * MW_THREADS;
      Ar[q][e] = q < nr && c < s ? a.G[(size_t)(wg + q * nwg) * s + c] : make_double2(0.0, 0.0);
    }
  }
  // the owned row slot of a column index (-1: not owned here)
  auto slot_of = [&](int c) {
    const int d = c - wg;
    return (d >= 0 && d % nwg == 0 && d / nwg < nr) ? d / nwg : -1;
  };
  // reflector J from its row x (valid from column J): v[c] for the own columns, tau returned;
  // row entries J and J+1 come from bcx (broadcast), the norm below J+1 from red_n
  auto reflector = [&](int J, const double2 x[EPT], double2 xj, double2 xj1, double xn2,
                       double2 v[EPT]) {
    const double2 alpha = cconj(xj1);
    double2 t = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
    double beta = alpha.x;
    if (!(xn2 == 0.0 && alpha.y == 0.0)) {
      const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
      beta = alpha.x >= 0.0 ? -nrm : nrm;
      const double ar = alpha.x - beta, ai = alpha.y;
      const double rb = 1.0 / beta, rden = 1.0 / (ar * ar + ai * ai);
      t = make_double2(-ar * rb, -ai * rb);
      scal = make_double2(ar * rden, -ai * rden);
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int c = tid + e * MW_THREADS;
      double2 val = make_double2(0.0, 0.0);
      if (c == J + 1) val = make_double2(1.0, 0.0);
      else if (c > J + 1 && c < s) val = cmul(cconj(x[e]), scal);
      v[e] = val;
      if (writer && c > J && c < s) W.V[(size_t)J * s + c] = val;
    }
    if (writer && tid == 0) {
      W.tau[J] = t;
      W.e[J] = beta;
      W.d[J] = xj.x;
    }
    return t;
  };
  double2 v[EPT], x[EPT];
  // reflector 0 from row 0
  double xn2 = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int c = tid + e * MW_THREADS;
    x[e] = c < s ? a.G[c] : make_double2(0.0, 0.0);
    if (c >= 2 && c < s) xn2 += x[e].x * x[e].x + x[e].y * x[e].y;
  }
  put_red_re(xn2, red_n);
  __syncthreads();
  double2 t = reflector(0, x, a.G[0], s > 1 ? a.G[1] : make_double2(0.0, 0.0),
                        sum_red_re<MW_WAVES>(red_n), v);
  // products of column 0 (rows r > 0), one pass over the rows
  auto products = [&](int j, const double2 vv[EPT]) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (q >= nr) break;
      double pr = 0.0, pi = 0.0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int c = tid + e * MW_THREADS;
        if (c > j && c < s) {
          const double2 av = Ar[q][e];
          pr += av.x * vv[e].x - av.y * vv[e].y;
          pi += av.x * vv[e].y + av.y * vv[e].x;
        }
      }
      pr = sum8(pr);
      pi = sum8(pi);
      if ((lane & 7) == 0) racc[q][wave * 8 + (lane >> 3)] = make_double2(pr, pi);
    }
  };
  auto publish_products = [&](int j) {
    // lanes 8q..8q+7 of wave 0 sum row q's 64 partials in a fixed order (eight each, then across
    // the eight lanes) and the first publishes y[r] for the rows r > j
    if (tid < 8 * nr) {
      const int q = tid >> 3, part = tid & 7;
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        yr += racc[q][part * 8 + i].x;
        yi += racc[q][part * 8 + i].y;
      }
      yr = sum8(yr);
      yi = sum8(yi);
      const int r = wg + q * nwg;
      if (part == 0 && r > j) cstore(&W.ybuf[(size_t)(j & 1) * s + r], make_double2(yr, yi));
    }
  };
  products(0, v);
  __syncthreads();
  publish_products(0);
  // phase times (tests only) accumulate in LDS, so that they take no registers of the other threads
  const bool stamp = a.tstamp && writer && tid == 0;
  __shared__ long long ph[8];
  if (stamp)
    for (int i = 0; i < 8; ++i) ph[i] = 0;
  auto lap = [&](int i) {
    if (stamp) {
      const long long t1 = wall_clock64();
      ph[i] += t1 - ph[7];
      ph[7] = t1;
    }
  };
  // with a tail, the reflectors from column s - tail on are left to the one-workgroup kernel
  const int jend = tail > 0 ? s - tail : s - 1;
  for (int j = 0; j < jend; ++j) {
    if (stamp) ph[7] = wall_clock64();
    // (1)
    if (!mw_sync(W.sync, nwg, (unsigned)(j + 1), &ok_sh, a.timeout_ticks)) {
      if (writer && tid == 0) W.d[0] = __builtin_nan("");
      if (tid == 0) raise_status(a.status, CBC_ETIMEOUT);
      return;
    }
    lap(0);
    // (2) everything published for this column, fetched at once into the own columns
    const double2* prev = j == 0 ? a.G + s : W.prow + (size_t)(j & 1) * s;
    double2 y[EPT], pv[EPT];
    double cr = 0.0, ci = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int c = tid + e * MW_THREADS;
      const bool in = c > j && c < s;
      y[e] = in ? cload(&W.ybuf[(size_t)(j & 1) * s + c]) : make_double2(0.0, 0.0);
      pv[e] = in ? (j == 0 ? prev[c] : cload(&prev[c])) : make_double2(0.0, 0.0);
      cr += v[e].x * y[e].x + v[e].y * y[e].y;     // conj(v) y
      ci += v[e].x * y[e].y - v[e].y * y[e].x;
      if (c == j + 1) bc[0] = y[e];
      const int q = slot_of(c);
      if (q >= 0) {
        ry[q] = y[e];
        rv[q] = v[e];
      }
    }
    put_red(cr, ci, red_c);
    __syncthreads();
    const double2 cs = sum_red(red_c);
    lap(1);
    // (3) w = tau y + a2 v with a2 = -|tau|^2 / 2 * conj(v^H y); row j+1 after the update
    const double tt = t.x * t.x + t.y * t.y;
    const double2 a2 = make_double2(-0.5 * tt * cs.x, 0.5 * tt * cs.y);
    double2 w[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const double2 ty = cmul(t, y[e]);
      w[e] = make_double2(ty.x + a2.x * v[e].x - a2.y * v[e].y, ty.y + a2.x * v[e].y + a2.y * v[e].x);
    }
    // v_j is 1 at j+1
    const double2 ty1 = cmul(t, bc[0]);
    const double2 w1 = make_double2(ty1.x + a2.x, ty1.y + a2.y);
    xn2 = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int c = tid + e * MW_THREADS;
      double2 xv = pv[e];
      // x -= v1 conj(w_c) + w1 conj(v_c), v1 = 1
      xv.x -= w[e].x + (w1.x * v[e].x + w1.y * v[e].y);
      xv.y -= -w[e].y + (w1.y * v[e].x - w1.x * v[e].y);
      x[e] = xv;
      if (c == j + 1) bc[1] = xv;
      if (c == j + 2) bc[2] = xv;
      if (c > j + 2 && c < s) xn2 += xv.x * xv.x + xv.y * xv.y;
    }
    put_red_re(xn2, red_n);
    __syncthreads();
    if (j + 1 >= s - 1) {
      // the last diagonal entry; no reflector, no further column
      if (writer && tid == 0) W.d[j + 1] = bc[1].x;
      break;
    }
    // the last column before the tail: the update only (no next reflector, no products)
    const bool last = j + 1 == jend;
    double2 vn[EPT];
    double2 t1 = make_double2(0.0, 0.0);
    if (last) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) vn[e] = make_double2(0.0, 0.0);
    } else {
      t1 = reflector(j + 1, x, bc[1], bc[2], sum_red_re<MW_WAVES>(red_n), vn);
    }
    lap(2);
    // (4) rank-2 update of the owned rows r > j+1 on the columns > j+1, the owner of row j+2
    // publishing it, and the products with v_{j+1} of the next column
    double2* pnext = W.prow + (size_t)((j + 1) & 1) * s;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (q >= nr) break;
      const int r = wg + q * nwg;
      double pr = 0.0, pi = 0.0;
      if (r > j + 1) {
        const double2 vr = rv[q];
        const double2 tyr = cmul(t, ry[q]);
        const double2 wr = make_double2(tyr.x + a2.x * vr.x - a2.y * vr.y,
                                        tyr.y + a2.x * vr.y + a2.y * vr.x);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int c = tid + e * MW_THREADS;
          if (c > j + 1 && c < s) {
            double2 xv = Ar[q][e];
            xv.x -= (vr.x * w[e].x + vr.y * w[e].y) + (wr.x * v[e].x + wr.y * v[e].y);
            xv.y -= (vr.y * w[e].x - vr.x * w[e].y) + (wr.y * v[e].x - wr.x * v[e].y);
            Ar[q][e] = xv;
            if (r == j + 2) cstore(&pnext[c], xv);
            pr += xv.x * vn[e].x - xv.y * vn[e].y;
            pi += xv.x * vn[e].y + xv.y * vn[e].x;
          }
        }
      }
      pr = sum8(pr);
      pi = sum8(pi);
      if ((lane & 7) == 0) racc[q][wave * 8 + (lane >> 3)] = make_double2(pr, pi);
    }
    __syncthreads();
    if (last) {
      // the trailing block (rows and columns from c0 = j + 1 = s - tail on) for the one-workgroup
      // kernel, densely with row stride `tail`, into G (whose rows every workgroup read at the
      // start): the rows' owners write their entries right of column c0; row c0 is the updated row
      // every workgroup holds in x, and workgroup 0 writes it and, conjugated, column c0 below it
      const int c0 = j + 1;
      double2* Tb = a.G;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int r = wg + q * nwg;
        if (q < nr && r > c0) {
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int c = tid + e * MW_THREADS;
            if (c > c0 && c < s) Tb[(size_t)(r - c0) * tail + (c - c0)] = Ar[q][e];
          }
        }
      }
      if (writer) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int c = tid + e * MW_THREADS;
          if (c >= c0 && c < s) {
            Tb[c - c0] = x[e];
            if (c > c0) Tb[(size_t)(c - c0) * tail] = cconj(x[e]);
          }
        }
      }
      break;
    }
    publish_products(j + 1);
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[e] = vn[e];
    t = t1;
    lap(3);
  }
  if (stamp) {
    // phases: 4 barrier, 5 fetch and v^H y, 6 the rest (8..9 its parts: next reflector, update
    // fused with the next products)
    a.tstamp[4] = ph[0];
    a.tstamp[5] = ph[1];
    a.tstamp[6] = ph[2] + ph[3];
    a.tstamp[8] = ph[2];
    a.tstamp[9] = ph[3];
  }
  if (writer && tail == 0) {
    __syncthreads();
    if (wave == 0) tri_bounds(W, s, a.tstamp, a.status);
  }
}

// the instantiation for EPT columns per thread with at least `rows` rows (nullptr: none)
static const void* mw_kernel(int ept, int rows) {
  if (ept == 1)
    return rows <= 1 ? (const void*)k_tridiag_mw<1, 1>
         : rows <= 2 ? (const void*)k_tridiag_mw<1, 2>
         : rows <= 3 ? (const void*)k_tridiag_mw<1, 3> : nullptr;
  if (ept == 2)
    return rows <= 3 ? (const void*)k_tridiag_mw<2, 3>
         : rows <= 4 ? (const void*)k_tridiag_mw<2, 4>
         : rows <= 5 ? (const void*)k_tridiag_mw<2, 5> : nullptr;
  if (ept == 3)
    return rows <= 5 ? (const void*)k_tridiag_mw<3, 5>
         : rows <= 6 ? (const void*)k_tridiag_mw<3, 6>
         : rows <= 7 ? (const void*)k_tridiag_mw<3, 7> : nullptr;
  return nullptr;
}

// ---- eigenvalues: one wave per eigenvalue -------------------------------------------------------
static constexpr int EV_WAVES = 4;

// The triangular factor of block b of the reflectors (one workgroup of 256 threads; run by extra
// workgroups of k_eigvals, which do not need it, so that it overlaps the eigenvalues: 0.18 ms at
// s = 1024 as a kernel of its own). The layout and use of the factors are described with k_bt_wy.
static constexpr int BT_CHUNK = 64;   // rows of a block staged in LDS for its Gram
__device__ void bt_tfactor_block(const EigArgs& a0, int b, int inst) {
  const EigArgs a = eig_inst(a0, inst);
  const int s = a.s, tid = threadIdx.x;
  EigWork W = eig_layout(a.work, s, a.kmax);
  const int j0 = b * BT_NB;
  const int n = s - 1 - j0 < BT_NB ? s - 1 - j0 : BT_NB;
  __shared__ double2 vs[BT_NB][BT_CHUNK + 1];
  __shared__ double2 G[BT_NB][BT_NB + 1];
  __shared__ double2 T[BT_NB][BT_NB + 1];
  // Gram entries G[p][q] = v_p^H v_q, p < q (nonzero rows: r > j0 + q), four entries per thread
  double2 acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = make_double2(0.0, 0.0);
  for (int r0 = j0 + 1; r0 < s; r0 += BT_CHUNK) {
    __syncthreads();
    for (int e = tid; e < BT_NB * BT_CHUNK; e += 256) {
      const int i = e / BT_CHUNK, l = e % BT_CHUNK, r = r0 + l, J = j0 + i;
      vs[i][l] = (i < n && r < s && r > J) ? W.V[(size_t)J * s + r] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int pq = tid + 256 * m, p = pq / BT_NB, q = pq % BT_NB;
      if (p < q && q < n) {
        double2 g = acc[m];
        for (int l = 0; l < BT_CHUNK; ++l) {
          const double2 x = vs[p][l], y = vs[q][l];
          g.x += x.x * y.x + x.y * y.y;
          g.y += x.x * y.y - x.y * y.x;
        }
        acc[m] = g;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int pq = tid + 256 * m, p = pq / BT_NB, q = pq % BT_NB;
    if (p < q && q < n) G[p][q] = acc[m];
  }
  __syncthreads();
  // row p of T in lane p, column by column (each lane reads only its own row of T)
  if (tid < BT_NB) {
    const int p = tid;
    for (int i = 0; i < BT_NB; ++i) {
      double2 v = make_double2(0.0, 0.0);
      if (i < n) {
        const double2 ti = W.tau[j0 + i];
        if (p == i) {
          v = ti;
        } else if (p < i) {
          double2 sm = make_double2(0.0, 0.0);
          for (int k = p; k < i; ++k) {
            const double2 c = cmul(T[p][k], G[k][i]);
            sm.x += c.x;
            sm.y += c.y;
          }
          const double2 c = cmul(ti, sm);
          v = make_double2(-c.x, -c.y);
        }
      }
      T[p][i] = v;
    }
    double2* dst = W.tfac + (size_t)b * BT_NB * BT_NB + (size_t)p * BT_NB;
    for (int i = 0; i < BT_NB; ++i) dst[i] = T[p][i];
  }
}

// With TF, the last bt_blocks(s) workgroups of the grid form the back-transformation's triangular
// factors instead (plain grids only).
template <bool TF>
__global__ __launch_bounds__(64 * EV_WAVES) void k_eigvals(EigArgs a0) {
  if (TF) {
    const int nev_wg = (int)gridDim.x - bt_blocks(a0.s);
    if ((int)blockIdx.x >= nev_wg) {
      bt_tfactor_block(a0, (int)blockIdx.x - nev_wg, blockIdx.y);
      return;
    }
  }
  if (!xcd_own(a0.spread)) return;
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
  // waves t < kmax: the kept candidates; t == kmax (if kmax < s): the next eigenvalue, for the gap
  // at the cut reported in the truncation record
  const int t = (int)(blockIdx.x / a0.spread) * EV_WAVES + wave;
  if (t > kmax || t >= s) return;
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
  if (lane == 0) {
    if (t < kmax) a.lam[t] = 0.5 * (lo + hi);
    else W.bounds[4] = 0.5 * (lo + hi);
  }
  if (a.tstamp && lane == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 2), (unsigned long long)wall_clock64());
}

// ---- eigenvectors of T and back-transformation: one wave per eigenpair ---------------------------
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Twisted factorisation T - x I = N_r Delta N_r^T for an isolated eigenvalue x, by a whole wave:
// every lane runs the recurrences (their values are the same in every lane), the coefficients of
// 64 consecutive steps are loaded one per lane and broadcast with readlane, and the result of step
// i is kept by lane i mod 64 and stored after each block of 64 steps. The operations and their
// order are those of the plain sequential recurrences. lp, dp, um, y: LDS scratch of s doubles
// each (y gets the unnormalised vector); returns 1 / ||y||.
__device__ double twisted_vector(const double* dd, const double* e, int s, double x, double pivmin,
                                 double* lp, double* dp, double* um, double* y) {
  const int lane = threadIdx.x & 63;
  // L+ D+ L+^T from the top
  double d = dd[0] - x;
  if (lane == 0) dp[0] = d;
  for (int i0 = 0; i0 < s - 1; i0 += 64) {
    const int il = i0 + lane;
    const double ddl = il + 1 < s ? dd[il + 1] : 0.0;
    const double el = il < s - 1 ? e[il] : 0.0;
    double lpl = 0.0, dpl = 0.0;
    const int nk = min(64, s - 1 - i0);
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      if (k < nk) {
        const double ddi = readlane_d(ddl, k), ei = readlane_d(el, k);
        if (fabs(d) < pivmin) d = d < 0.0 ? -pivmin : pivmin;
        const double l = qdiv(ei, d);
        d = ddi - x - l * ei;
        if (lane == k) {
          lpl = l;
          dpl = d;
        }
      }
    }
    if (il < s - 1) {
      lp[il] = lpl;
      dp[il + 1] = dpl;
    }
  }
  wave_lds_sync();
  // U- D- U-^T from the bottom, and the twist index r of the smallest |gamma|
  double dm = dd[s - 1] - x;
  int r = s - 1;
  double gbest = fabs(dp[s - 1]);
  for (int i1 = s - 2; i1 >= 0; i1 -= 64) {
    const int il = i1 - lane;
    const double ddl = il >= 0 ? dd[il] : 0.0, el = il >= 0 ? e[il] : 0.0, dpl = il >= 0 ? dp[il] : 0.0;
    double uml = 0.0;
    const int nk = min(64, i1 + 1);
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      if (k < nk) {
        const double ddi = readlane_d(ddl, k), ei = readlane_d(el, k), dpi = readlane_d(dpl, k);
        if (fabs(dm) < pivmin) dm = dm < 0.0 ? -pivmin : pivmin;
        const double u = qdiv(ei, dm);
        dm = ddi - x - u * ei;
        const double g = fabs(dpi + dm - (ddi - x));
        if (g < gbest) {
          gbest = g;
          r = i1 - k;
        }
        if (lane == k) uml = u;
      }
    }
    if (il >= 0) um[il] = uml;
  }
  wave_lds_sync();
  // y[r] = 1, y[i] = -lp[i] y[i+1] below r, y[i+1] = -um[i] y[i] above
  double z = 1.0, nrm = 1.0;
  if (lane == 0) y[r] = 1.0;
  for (int i1 = r - 1; i1 >= 0; i1 -= 64) {
    const int il = i1 - lane;
    const double lpl = il >= 0 ? lp[il] : 0.0;
    double yl = 0.0;
    const int nk = min(64, i1 + 1);
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      if (k < nk) {
        z = -readlane_d(lpl, k) * z;
        nrm += z * z;
        if (lane == k) yl = z;
      }
    }
    if (il >= 0) y[il] = yl;
  }
  z = 1.0;
  for (int i0 = r; i0 < s - 1; i0 += 64) {
    const int il = i0 + lane;
    const double uml = il < s - 1 ? um[il] : 0.0;
    double yl = 0.0;
    const int nk = min(64, s - 1 - i0);
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      if (k < nk) {
        z = -readlane_d(uml, k) * z;
        nrm += z * z;
        if (lane == k) yl = z;
      }
    }
    if (il < s - 1) y[il + 1] = yl;
  }
  wave_lds_sync();
  return 1.0 / sqrt(nrm);
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

// Register-resident variant for s <= 64 R: lane l holds rows l + 64 q. The next PF reflectors and
// their tau are held in registers, loaded PF steps before their use, so that the L2 latency of a
// reflector overlaps PF reductions.
template <int R, int PF>
__device__ void back_transform_reg(const EigArgs& a, const EigWork& W, int s, int kmax, int t,
                                   bool kept, const double* yin) {
  const int lane = threadIdx.x & 63;
  double2 ur[R], vn[PF][R], tn[PF];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = lane + 64 * q;
    ur[q] = make_double2(i < s ? yin[i] : 0.0, 0.0);
  }
  auto fetch = [&](int j, double2& tau, double2* v) {
    tau = j >= 0 ? W.tau[j] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = lane + 64 * q;
      v[q] = (j >= 0 && i > j && i < s) ? W.V[(size_t)j * s + i] : make_double2(0.0, 0.0);
    }
  };
#pragma unroll
  for (int p = 0; p < PF; ++p) fetch(s - 2 - p, tn[p], vn[p]);
  for (int j0 = s - 2; j0 >= 0; j0 -= PF) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int j = j0 - p;
      if (j < 0) break;
      double2 vc[R];
#pragma unroll
      for (int q = 0; q < R; ++q) vc[q] = vn[p][q];
      const double2 tc = tn[p];
      fetch(j - PF, tn[p], vn[p]);
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
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = lane + 64 * q;
    if (i < s) a.U[(size_t)i * kmax + t] = kept ? ur[q] : make_double2(0.0, 0.0);
  }
}

// ---- eigenvectors: three launches ----------------------------------------------------------------
// (A) one wave per eigenpair: the twisted-factorisation eigenvector of T, to Y;
// (B) one wave per cluster of close eigenvalues: modified Gram-Schmidt of the members in order
//     (or inverse iteration for near-exact degeneracies), in place in Y;
// (C) one wave per eigenpair: back-transformation u = Q y with the vector held in registers.
// Separating (A) and (C) from (B) keeps the twisted solves and the back-transformations parallel
// over all eigenpairs even where eigenvalues fall into clusters (measured at s = 128: 107 us
// without clusters, 280 us with three clusters, where one wave per cluster doing all of its
// members' work took 1374 us).

__device__ inline int keep_count(const EigArgs& a) {
  int keep = a.kmax;
  if (a.tol > 0.0) {
    const double cut = a.tol * a.tol * a.lam[0];
    int c = 0;
    for (int u = threadIdx.x & 63; u < a.kmax; u += 64) c += a.lam[u] > cut;
    c = (int)wave_sum((double)c);
    keep = c < 1 ? 1 : c;
  }
  return keep;
}
// u starts a cluster: its gap to the previous eigenvalue exceeds 1e-3 ||T||, or it is negligible
__device__ inline bool cluster_start(const double* lam, int u, int kmax, double tnorm) {
  const double ortol = 1e-3 * tnorm, tiny = 64.0 * DBL_EPSILON * tnorm;
  return u == 0 || u == kmax || lam[u - 1] - lam[u] > ortol || lam[u] <= tiny;
}

__global__ __launch_bounds__(256) void k_eigvecs_twisted(EigArgs a0) {
  if (!xcd_own(a0.spread)) return;
  const EigArgs a = eig_inst(a0, blockIdx.y);
  extern __shared__ double smem[];
  const int s = a.s, kmax = a.kmax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  double* dd = smem;
  double* el = dd + s;
  double* region = el + s + 4 * (size_t)s * wave;   // per wave: lp | dp | um | y
  EigWork W = eig_layout(a.work, s, kmax);
  for (int i = tid; i < s; i += blockDim.x) {
    dd[i] = W.d[i];
    el[i] = i < s - 1 ? W.e[i] : 0.0;
  }
  __syncthreads();
  const int t = (int)(blockIdx.x / a0.spread) * nw + wave;
  if (t >= kmax) return;
  const int keep = keep_count(a);
  if (t == 0 && lane == 0) {
    a.kkeep[0] = keep;
    a.inv_sqrt_l0[0] = a.lam[0] > 0.0 ? 1.0 / sqrt(a.lam[0]) : 1.0;
  }
  if (t == 0 && a.rec) {
    // the truncation record: discarded weight (trace of T minus the kept eigenvalues) and the
    // relative gap at the cut
    double tr = 0.0, kept = 0.0;
    for (int i = lane; i < s; i += 64) tr += dd[i];
    for (int u = lane; u < keep; u += 64) kept += a.lam[u];
    tr = wave_sum(tr);
    kept = wave_sum(kept);
    if (lane == 0) {
      const bool cut = keep < s;
      const double next = keep < kmax ? a.lam[keep] : (cut ? W.bounds[4] : 0.0);
      const double last = a.lam[keep - 1];
      const double gap = !cut ? 1.0 : (last > 0.0 ? (last - next) / last : 0.0);
      cbc_trunc_record r;
      r.node = a.rec_node;
      r.sweep = a.rec_sweep;
      r.dim = s;
      r.kmax = kmax;
      r.kept = keep;
      r.flags = gap < 1e-8 ? 1 : 0;
      r.discarded = tr > 0.0 ? fmax(0.0, (tr - kept) / tr) : 0.0;
      r.gap = gap;
      *a.rec = r;
      if (!isfinite(tr)) raise_status(a.status, CBC_ENOTPD);
    }
  }
  double* y = region + 3 * (size_t)s;
  const double inv = twisted_vector(dd, el, s, a.lam[t], W.bounds[3], region, region + s, region + 2 * s, y);
  double* yo = W.Y + (size_t)t * s;
  for (int i = lane; i < s; i += 64) yo[i] = y[i] * inv;
}

__global__ __launch_bounds__(256) void k_eigvecs_clusters(EigArgs a0) {
  if (!xcd_own(a0.spread)) return;
  const EigArgs a = eig_inst(a0, blockIdx.y);
  extern __shared__ double smem[];
  const int s = a.s, kmax = a.kmax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  EigWork W = eig_layout(a.work, s, kmax);
  const int t = (int)(blockIdx.x / a0.spread) * nw + wave;
  if (t >= kmax) return;
  const double tnorm = W.bounds[2];
  const double* lam = a.lam;
  if (!cluster_start(lam, t, kmax, tnorm)) return;
  int ce = t + 1;
  while (ce < kmax && !cluster_start(lam, ce, kmax, tnorm)) ++ce;
  if (ce == t + 1) return;
  if (a.tstamp && lane == 0) atomicAdd(reinterpret_cast<unsigned long long*>(a.tstamp + 7), 1ull);
  double mingap = DBL_MAX;
  for (int m = t + 1; m < ce; ++m) mingap = fmin(mingap, lam[m - 1] - lam[m]);
  if (mingap > 1e-12 * tnorm) {
    // twisted vectors are accurate up to mixing inside the cluster: two passes of modified
    // Gram-Schmidt over the members in order give an orthonormal basis of its invariant subspace
    for (int m = t + 1; m < ce; ++m) {
      double* ym = W.Y + (size_t)m * s;
      for (int pass = 0; pass < 2; ++pass) {
        for (int q = t; q < m; ++q) {
          const double* yq = W.Y + (size_t)q * s;
          double dot = 0.0;
          for (int i = lane; i < s; i += 64) dot += yq[i] * ym[i];
          dot = wave_sum(dot);
          for (int i = lane; i < s; i += 64) ym[i] -= dot * yq[i];
        }
      }
      double nrm = 0.0;
      for (int i = lane; i < s; i += 64) nrm += ym[i] * ym[i];
      nrm = wave_sum(nrm);
      const double inv = 1.0 / sqrt(nrm);
      for (int i = lane; i < s; i += 64) ym[i] *= inv;
    }
  } else {
    double* dd = smem + 2 * (size_t)s * wave;
    double* el = dd + s;
    for (int i = lane; i < s; i += 64) {
      dd[i] = W.d[i];
      el[i] = i < s - 1 ? W.e[i] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) cluster_vectors(dd, el, s, lam, t, ce, tnorm, W.Y, W.lu + (size_t)t * 5 * s);
  }
}

// one instantiation per size class, so that small matrices run with few registers per wave (many
// waves per SIMD when instances are batched)
template <int R, int PF>
__global__ __launch_bounds__(256) void k_backtransform(EigArgs a0) {
  if (!xcd_own(a0.spread)) return;
  const EigArgs a = eig_inst(a0, blockIdx.y);
  extern __shared__ double smem[];
  const int s = a.s, kmax = a.kmax;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  EigWork W = eig_layout(a.work, s, kmax);
  const int t = (int)(blockIdx.x / a0.spread) * nw + wave;
  if (t >= kmax) return;
  const bool kept = t < a.kkeep[0];
  const double* y = W.Y + (size_t)t * s;
  if (R > 0) back_transform_reg<(R > 0 ? R : 1), PF>(a, W, s, kmax, t, kept, y);
  else back_transform_col(a, W, s, kmax, t, kept, y, reinterpret_cast<double2*>(smem) + (size_t)s * wave);
  if (a.tstamp && (threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 3), (unsigned long long)wall_clock64());
}

// ---- blocked back-transformation (s > 256): compact WY, u = Q y with Q = B_0 B_1 ... B_{nb-1} ------
// Block b holds the reflectors j0 = BT_NB b ... j0 + n - 1 and equals I - V_b T_b V_b^H with T_b upper
// triangular: T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] (V_b[:, 0:i]^H v_i). The factors are formed
// once per solve (bt_tfactor_block, one workgroup per block); k_bt_wy then applies the blocks, last one
// first, to CPW eigenvectors per workgroup held in LDS: w = V_b^H x, w' = T_b w, x -= V_b w'. Each
// block costs one dependent step instead of BT_NB reflector-by-reflector reductions, and the
// reflectors are read with unit stride in both passes. Measured on MI355X (eigenvectors of T and
// back-transformation, k = 256): s = 1024 1.62 -> 0.83 ms, 1272 5.4 -> 1.15, 1536 7.75 -> 1.52
// against one wave per eigenvector applying the reflectors one at a time; one eigenvector per
// workgroup (256 workgroups) was faster than two (0.91 ms at s = 1024).
static constexpr int BT_CPW = 1;      // eigenvectors per workgroup of k_bt_wy
static constexpr int BT_THREADS = 512; // threads per workgroup of k_bt_wy


template <int CPW>   // eigenvectors per workgroup
__global__ __launch_bounds__(BT_THREADS) void k_bt_wy(EigArgs a0) {
  const EigArgs a = eig_inst(a0, blockIdx.y);
  const int s = a.s, kmax = a.kmax, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  EigWork W = eig_layout(a.work, s, kmax);
  const int t0 = blockIdx.x * CPW;
  extern __shared__ double smem[];
  double2* X = reinterpret_cast<double2*>(smem);   // X[r * CPW + c]
  __shared__ double2 Ws[BT_NB][CPW], Wq[BT_NB][CPW];
  for (int e = tid; e < s * CPW; e += BT_THREADS) {
    const int r = e / CPW, t = t0 + e % CPW;
    X[e] = make_double2(t < kmax ? W.Y[(size_t)t * s + r] : 0.0, 0.0);
  }
  __syncthreads();
  constexpr int NWV = BT_THREADS / 64;
  constexpr int PW = BT_NB / NWV;   // reflectors per wave in the first pass
  for (int b = bt_blocks(s) - 1; b >= 0; --b) {
    const int j0 = b * BT_NB;
    const int n = s - 1 - j0 < BT_NB ? s - 1 - j0 : BT_NB;
    // (1) w = V_b^H x: wave w takes the reflectors w, w + NWV, ...; lanes run over the rows
    double2 acc[PW][CPW];
#pragma unroll
    for (int m = 0; m < PW; ++m)
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[m][c] = make_double2(0.0, 0.0);
#pragma unroll 2
    for (int r = j0 + 1 + lane; r < s; r += 64) {
      // loads issued together from in-bounds addresses (reflector index clamped to s - 2); the
      // entries outside a reflector's support are replaced by zeros below
      double2 vv[PW];
#pragma unroll
      for (int m = 0; m < PW; ++m) {
        const int J = j0 + wave + NWV * m;
        vv[m] = W.V[(size_t)(J < s - 1 ? J : s - 2) * s + r];
      }
      double2 x[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) x[c] = X[r * CPW + c];
#pragma unroll
      for (int m = 0; m < PW; ++m) {
        const int i = wave + NWV * m;
        const double2 v = (i < n && r > j0 + i) ? vv[m] : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          acc[m][c].x += v.x * x[c].x + v.y * x[c].y;
          acc[m][c].y += v.x * x[c].y - v.y * x[c].x;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < PW; ++m)
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const double re = wave_sum(acc[m][c].x), im = wave_sum(acc[m][c].y);
        if (lane == 0) Ws[wave + NWV * m][c] = make_double2(re, im);
      }
    __syncthreads();
    // (2) w' = T_b w (T_b is zero outside the block's n x n upper triangle)
    if (tid < BT_NB * CPW) {
      const int i = tid / CPW, c = tid % CPW;
      const double2* trow = W.tfac + (size_t)b * BT_NB * BT_NB + (size_t)i * BT_NB;
      double2 tr[BT_NB];
#pragma unroll
      for (int k = 0; k < BT_NB; ++k) tr[k] = trow[k];
      double2 sm = make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < BT_NB; ++k) {
        const double2 p = cmul(tr[k], Ws[k][c]);
        sm.x += p.x;
        sm.y += p.y;
      }
      Wq[i][c] = sm;
    }
    __syncthreads();
    // (3) x -= V_b w', one row per thread; the block's reflectors at the row are loaded together,
    // half a block at a time
    for (int r = j0 + 1 + tid; r < s; r += BT_THREADS) {
      const int imax = r - j0 < n ? r - j0 : n;   // reflector i is nonzero at row r iff r > j0 + i
      double2 u[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) u[c] = make_double2(0.0, 0.0);
#pragma unroll
      for (int h = 0; h < BT_NB; h += BT_NB / 2) {
        double2 vv[BT_NB / 2];
#pragma unroll
        for (int i = 0; i < BT_NB / 2; ++i) {
          const int J = j0 + h + i;
          vv[i] = W.V[(size_t)(J < s - 1 ? J : s - 2) * s + r];
        }
#pragma unroll
        for (int i = 0; i < BT_NB / 2; ++i)
          if (h + i >= imax) vv[i] = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < BT_NB / 2; ++i) {
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            const double2 p = cmul(vv[i], Wq[h + i][c]);
            u[c].x += p.x;
            u[c].y += p.y;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        X[r * CPW + c].x -= u[c].x;
        X[r * CPW + c].y -= u[c].y;
      }
    }
    __syncthreads();
  }
  const int kk = a.kkeep[0];
  for (int e = tid; e < s * CPW; e += BT_THREADS) {
    const int r = e / CPW, t = t0 + e % CPW;
    if (t < kmax) a.U[(size_t)r * kmax + t] = t < kk ? X[e] : make_double2(0.0, 0.0);
  }
  if (a.tstamp && tid == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.tstamp + 3), (unsigned long long)wall_clock64());
}

size_t eig_lds_bytes(int s) { return (size_t)16 * (s * (size_t)(s + 1) / 2) + (size_t)s * (3 * 16) + 64; }

hipError_t launch_eig(const EigArgs& a0, hipStream_t st) {
  if (a0.s <= 0 || a0.kmax <= 0 || a0.kmax > a0.s || a0.batch <= 0) return hipErrorInvalidValue;
  EigArgs a = a0;
  a.spread = a.s <= 256 && a.batch < XCD_SPREAD ? XCD_SPREAD : 1;
  if (!eig_size_supported(a.s) || (a.s > EIG_LDS_MAX && a.reduction == 1 && !mw_size_supported(a.s)))
    return hipErrorInvalidValue;
  const bool two_stage = a.s > EIG_LDS_MAX && a.reduction == 0;
  if (a.s <= EIG_LDS_MAX) {
    const size_t lds = eig_lds_bytes(a.s);
    (void)hipFuncSetAttribute((const void*)k_tridiag, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k_tridiag, dim3(a.batch), dim3(EIG_THREADS), lds, st, a, a.s);
  } else if (two_stage) {
    const hipError_t z = launch_band_reduction(a, st);
    if (z != hipSuccess) return z;
  } else {
    const MwShape m = mw_shape(a.s);
    if (!mw_size_supported(a.s)) return hipErrorInvalidValue;
    // the barrier words start at zero for every call
    EigWork W = eig_layout(a.work, a.s, a.kmax);
    hipError_t z = launch_zero(W.sync, MW_SYNC_BYTES, a.batch, a.bs, st);
    if (z != hipSuccess) return z;
    // columns per thread and rows per workgroup: the smallest instantiation that covers both
    const void* fn = mw_kernel((a.s + MW_THREADS - 1) / MW_THREADS, m.rows);
    if (!fn) return hipErrorInvalidValue;
    // its workgroups wait for each other: no other such solve may hold compute units meanwhile
    z = mw_gate_enter(st);
    if (z != hipSuccess) return z;
    EigArgs ka = a;
    int knwg = m.nwg, ktail = MW_TAIL;
    void* kargs[] = {(void*)&ka, (void*)&knwg, (void*)&ktail};
    z = hipLaunchKernel(fn, dim3(m.nwg, a.batch), dim3(MW_THREADS), kargs, 0, st);
    if (z != hipSuccess) return z;
    z = hipGetLastError();
    if (z != hipSuccess) return z;
    z = mw_gate_leave(st);
    if (z != hipSuccess) return z;
    // the last MW_TAIL columns in one workgroup, from the block the reduction left in G
    EigArgs ta = a;
    ta.s = MW_TAIL;
    const size_t tlds = eig_lds_bytes(MW_TAIL);
    (void)hipFuncSetAttribute((const void*)k_tridiag, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)tlds);
    hipLaunchKernelGGL(k_tridiag, dim3(a.batch), dim3(EIG_THREADS), tlds, st, ta, a.s);
    z = hipGetLastError();
    if (z != hipSuccess) return z;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds2 = (size_t)16 * a.s;
  const int nev = a.kmax < a.s ? a.kmax + 1 : a.kmax;
  // the blocked back-transformation's factors are formed by extra workgroups of this launch
  const bool blocked_bt = !two_stage && a.s > 256 && a.spread == 1;
  const unsigned nev_wg = (unsigned)(a.spread * ((nev + EV_WAVES - 1) / EV_WAVES));
  if (blocked_bt)
    hipLaunchKernelGGL(k_eigvals<true>, dim3(nev_wg + bt_blocks(a.s), a.batch), dim3(64 * EV_WAVES),
                       lds2, st, a);
  else
    hipLaunchKernelGGL(k_eigvals<false>, dim3(nev_wg, a.batch), dim3(64 * EV_WAVES), lds2, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nw = a.s <= 1000 ? 4 : (a.s <= 1900 ? 2 : 1);
  const size_t lds3 = (size_t)a.s * (2 * 8 + (size_t)nw * 4 * 8) + 64;
  if (lds3 > 160 * 1024 - 512) return hipErrorInvalidValue;
  const dim3 g3(a.spread * ((a.kmax + nw - 1) / nw), a.batch);
  (void)hipFuncSetAttribute((const void*)k_eigvecs_twisted,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds3);
  hipLaunchKernelGGL(k_eigvecs_twisted, g3, dim3(64 * nw), lds3, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t ldsc = (size_t)a.s * 2 * 8 * 4;
  if (ldsc > 160 * 1024 - 512) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)k_eigvecs_clusters,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsc);
  hipLaunchKernelGGL(k_eigvecs_clusters, dim3(a.spread * ((a.kmax + 3) / 4), a.batch), dim3(256),
                     ldsc, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (two_stage) return launch_bt_band(a, st);
  const dim3 gb(a.spread * ((a.kmax + 3) / 4), a.batch);
  if (blocked_bt) {
    const size_t ldsx = (size_t)a.s * BT_CPW * 16;
    if (ldsx > 160 * 1024 - 8192) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute((const void*)k_bt_wy<BT_CPW>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsx);
    hipLaunchKernelGGL(k_bt_wy<BT_CPW>, dim3((a.kmax + BT_CPW - 1) / BT_CPW, a.batch),
                       dim3(BT_THREADS), ldsx, st, a);
  } else if (a.s <= 64) {
    hipLaunchKernelGGL((k_backtransform<1, 4>), gb, dim3(256), 0, st, a);
  } else if (a.s <= 128) {
    hipLaunchKernelGGL((k_backtransform<2, 4>), gb, dim3(256), 0, st, a);
  } else if (a.s <= 256) {
    hipLaunchKernelGGL((k_backtransform<4, 4>), gb, dim3(256), 0, st, a);
  } else if (a.s <= 512) {
    hipLaunchKernelGGL((k_backtransform<8, 2>), gb, dim3(256), 0, st, a);
  } else if (a.s <= 1024) {
    hipLaunchKernelGGL((k_backtransform<16, 1>), gb, dim3(256), 0, st, a);
  } else {
    const size_t ldsb = (size_t)a.s * 16 * 4;
    if (ldsb > 160 * 1024 - 512) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute((const void*)k_backtransform<0, 1>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsb);
    hipLaunchKernelGGL((k_backtransform<0, 1>), gb, dim3(256), ldsb, st, a);
  }
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
  if (!isfinite(lam[0])) {
    // a failed eigensolve: the output must not look like a valid (zero) environment
    out = make_double2(__builtin_nan(""), __builtin_nan(""));
  } else if (j < kkeep[0] && lam[0] > 0.0) {
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
