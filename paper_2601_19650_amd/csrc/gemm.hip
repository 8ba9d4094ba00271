// Complex tensor-contraction GEMM on gfx950 matrix cores.
//
// Every contraction of the compression sweeps (environment absorption, operator contraction, Gram
// matrices, projections and environment updates) is one call of this kernel: rows, columns and
// reduction indices are multi-indices over tensor legs, mapped to element offsets through small
// device tables, so no transposes are ever materialised.
//
// Complex products are carried by real MFMA products on planar tiles:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B
// FP32 accumulation uses v_mfma_f32_16x16x4_f32, FP64 accumulation v_mfma_f64_16x16x4_f64. Tiles
// are staged in LDS as k-major planar arrays so every lane's MFMA operand read is contiguous.
#include "cbc_internal.h"

namespace cbc {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T> struct Acc4;
template <> struct Acc4<float> { using type = f4v; };
template <> struct Acc4<double> { using type = d4v; };

__device__ __forceinline__ f4v mfma16(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// C tile BM x BN per workgroup of 4 waves (2 x 2), each wave (BM/2) x (BN/2) in 16 x 16 blocks.
template <typename TA, typename TB, typename TC, typename ACC, int BM, int BN>
__global__ __launch_bounds__(256) void k_cgemm(GemmArgs g) {
  constexpr int BK = sizeof(ACC) == 8 ? 8 : 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int MB = WM / 16, NB = WN / 16;
  constexpr int PAD = sizeof(ACC) == 8 ? 1 : 4;
  using CA = typename Cplx<TA>::type;
  using CB = typename Cplx<TB>::type;
  using CC = typename Cplx<TC>::type;
  using V4 = typename Acc4<ACC>::type;

  __shared__ ACC sAr[BK][BM + PAD];
  __shared__ ACC sAi[BK][BM + PAD];
  __shared__ ACC sBr[BK][BN + PAD];
  __shared__ ACC sBi[BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int m0 = g.mbase + blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;
  const int M = g.M, N = g.N;
  const int bz = blockIdx.z / g.ksplit, kz = blockIdx.z % g.ksplit;
  const int kbeg = g.ksplit > 1 ? kz * g.kchunk : 0;
  const int K = g.ksplit > 1 ? min(g.K, kbeg + g.kchunk) : g.K;
  // a Hermitian product computes the tiles on and below the diagonal only (BM == BN)
  if (g.herm && n0 >= m0 + BM) return;
  if (g.skip && *inst_ptr(g.skip, g.bsSkip, bz)) return;
  const CA* __restrict__ A = reinterpret_cast<const CA*>(inst_ptr(g.A, g.bsA, bz));
  const CB* __restrict__ B = reinterpret_cast<const CB*>(inst_ptr(g.B, g.bsB, bz));
  const ACC sa = g.conjA ? ACC(-1) : ACC(1);
  const ACC sb = g.conjB ? ACC(-1) : ACC(1);

  V4 accr[MB][NB], acci[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      accr[i][j] = V4{0, 0, 0, 0};
      acci[i][j] = V4{0, 0, 0, 0};
    }

  for (int k0 = kbeg; k0 < K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int r, kk;
      if (g.a_kfast) { kk = e % BK; r = e / BK; } else { r = e % BM; kk = e / BM; }
      const int m = m0 + r, k = k0 + kk;
      ACC re = 0, im = 0;
      if (m < M && k < K) {
        const CA v = A[g.offAm ? (int64_t)g.offAm[m] + g.offAk[k] : m * g.sAm + k * g.sAk];
        re = ACC(v.x);
        im = sa * ACC(v.y);
      }
      sAr[kk][r] = re;
      sAi[kk][r] = im;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int c, kk;
      if (g.b_kfast) { kk = e % BK; c = e / BK; } else { c = e % BN; kk = e / BN; }
      const int n = n0 + c, k = k0 + kk;
      ACC re = 0, im = 0;
      if (n < N && k < K) {
        const CB v = B[g.offAm ? (int64_t)g.offBk[k] + g.offBn[n] : k * g.sBk + n * g.sBn];
        re = ACC(v.x);
        im = sb * ACC(v.y);
      }
      sBr[kk][c] = re;
      sBi[kk][c] = im;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      ACC ar[MB], ai[MB], br[NB], bi[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        ar[i] = sAr[kr][wr * WM + i * 16 + (lane & 15)];
        ai[i] = sAi[kr][wr * WM + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        br[j] = sBr[kr][wc * WN + j * 16 + (lane & 15)];
        bi[j] = sBi[kr][wc * WN + j * 16 + (lane & 15)];
      }
      // the two products into each accumulator are issued a full sweep apart, so dependent MFMAs
      // never follow each other
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accr[i][j] = mfma16(ar[i], br[j], accr[i][j]);
          acci[i][j] = mfma16(ar[i], bi[j], acci[i][j]);
        }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accr[i][j] = mfma16(-ai[i], bi[j], accr[i][j]);
          acci[i][j] = mfma16(ai[i], br[j], acci[i][j]);
        }
    }
    __syncthreads();
  }

  if (g.ksplit > 1) {
    // raw chunk sums, row-major M x N per (instance, chunk)
    using CP = typename Cplx<ACC>::type;
    CP* __restrict__ P = reinterpret_cast<CP*>(inst_ptr(g.part, g.bsPart, bz)) + (int64_t)kz * M * N;
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int n = n0 + wc * WN + j * 16 + (lane & 15);
        if (n >= N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rb = sizeof(ACC) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
          const int m = m0 + wr * WM + i * 16 + rb;
          if (m < M) P[(int64_t)m * N + n] = CP{accr[i][j][r], acci[i][j][r]};
        }
      }
    return;
  }
  double alpha = g.alpha;
  if (g.alpha_dev) alpha *= inst_ptr(g.alpha_dev, g.bsAlpha, bz)[0];
  if (g.alpha_dev2) alpha *= inst_ptr(g.alpha_dev2, g.bsAlpha2, bz)[0];
  CC* __restrict__ C = reinterpret_cast<CC*>(inst_ptr(g.C, g.bsC, bz));
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wc * WN + j * 16 + (lane & 15);
      if (n >= N) continue;
      const int64_t cn = g.offAm ? (int64_t)g.offCn[n] : n * g.sCn;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // output rows of a 16x16 block: FP32 MFMA lane l, register r -> row 4*(l/16) + r;
        // FP64 MFMA -> row l/16 + 4*r (column l%16 in both)
        const int rb = sizeof(ACC) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int m = m0 + wr * WM + i * 16 + rb;
        if (m < M && (!g.herm || m >= n)) {
          const int64_t ci = (g.offAm ? (int64_t)g.offCm[m] : m * g.sCm) + cn;
          double xr = double(accr[i][j][r]) * alpha, xi = double(acci[i][j][r]) * alpha;
          if (g.accum) {
            const CC old = C[ci];
            xr += double(old.x);
            xi += double(old.y);
          }
          CC out;
          out.x = TC(xr);
          out.y = TC(xi);
          C[ci] = out;
          if (g.herm && m > n) {
            out.y = -out.y;
            C[(g.offAm ? (int64_t)g.offCm[n] + g.offCn[m] : n * g.sCm + m * g.sCn)] = out;
          }
        }
      }
    }
}

// Second pass of a split-K GEMM: C = alpha * sum over the chunks, in chunk order.
template <typename TC, typename ACC>
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs g) {
  using CP = typename Cplx<ACC>::type;
  using CC = typename Cplx<TC>::type;
  const int b = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)g.M * g.N;
  if (idx >= mn) return;
  if (g.skip && *inst_ptr(g.skip, g.bsSkip, b)) return;
  const int m = (int)(idx / g.N), n = (int)(idx % g.N);
  // a Hermitian product has chunk sums on and below the diagonal only: (m, n) above it is the
  // conjugate of (n, m)
  const bool mirror = g.herm && m < n;
  const CP* P = reinterpret_cast<const CP*>(inst_ptr(g.part, g.bsPart, b)) +
                (mirror ? (int64_t)n * g.N + m : idx);
  double re = 0.0, im = 0.0;
  for (int z = 0; z < g.ksplit; ++z) {
    const CP v = P[(int64_t)z * mn];
    re += double(v.x);
    im += double(v.y);
  }
  if (mirror) im = -im;
  double alpha = g.alpha;
  if (g.alpha_dev) alpha *= inst_ptr(g.alpha_dev, g.bsAlpha, b)[0];
  if (g.alpha_dev2) alpha *= inst_ptr(g.alpha_dev2, g.bsAlpha2, b)[0];
  CC* C = reinterpret_cast<CC*>(inst_ptr(g.C, g.bsC, b));
  const int64_t ci = g.offAm ? (int64_t)g.offCm[m] + g.offCn[n] : m * g.sCm + n * g.sCn;
  double xr = re * alpha, xi = im * alpha;
  if (g.accum) {
    const CC old = C[ci];
    xr += double(old.x);
    xi += double(old.y);
  }
  CC out;
  out.x = TC(xr);
  out.y = TC(xi);
  C[ci] = out;
}

// Pipelined variant with 64 x 64 tiles (BK = 16 with FP32 accumulation, 8 with FP64): the row /
// column offsets of the tile are read once into registers, the next k-tile is fetched from global
// memory into registers while the MFMAs consume the current one from LDS, and the LDS tiles are
// double-buffered so each k-tile costs one barrier. A Hermitian product (g.herm) computes the tiles
// on and below the diagonal and writes each strictly lower entry also, conjugated, at its mirror.
template <typename TA, typename TB, typename TC, typename ACC, int BM, int BN, int WGM = 2,
          int WGN = 2>
__device__ __forceinline__ void cgemm_pipe_body(const GemmArgs& g) {
  constexpr bool F64 = sizeof(ACC) == 8;
  constexpr int NT = 64 * WGM * WGN;                       // threads: a WGM x WGN grid of waves
  constexpr int BK = (F64 || BM * BN > 64 * 64) ? 8 : 16;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int MB = WM / 16, NB = WN / 16;
  constexpr int PAD = F64 ? 1 : 4;
  constexpr int EA = BM * BK / NT, EB = BN * BK / NT;     // elements per thread and k-tile
  static_assert(EA * NT == BM * BK && EB * NT == BN * BK, "tile loads must divide evenly");
  using CA = typename Cplx<TA>::type;
  using CB = typename Cplx<TB>::type;
  using CC = typename Cplx<TC>::type;
  using V4 = typename Acc4<ACC>::type;

  __shared__ ACC sAr[2][BK][BM + PAD];
  __shared__ ACC sAi[2][BK][BM + PAD];
  __shared__ ACC sBr[2][BK][BN + PAD];
  __shared__ ACC sBi[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WGN, wc = wave % WGN;
  const int m0 = g.mbase + blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;
  if (g.herm && n0 >= m0 + BM) return;   // strictly above the diagonal (BM == BN)
  const int M = g.M, N = g.N;
  const int bz = blockIdx.z / g.ksplit, kz = blockIdx.z % g.ksplit;
  if (g.skip && *inst_ptr(g.skip, g.bsSkip, bz)) return;
  const int kbeg = g.ksplit > 1 ? kz * g.kchunk : 0;
  const int K = g.ksplit > 1 ? min(g.K, kbeg + g.kchunk) : g.K;
  const CA* __restrict__ A = reinterpret_cast<const CA*>(inst_ptr(g.A, g.bsA, bz));
  const CB* __restrict__ B = reinterpret_cast<const CB*>(inst_ptr(g.B, g.bsB, bz));
  const ACC sa = g.conjA ? ACC(-1) : ACC(1);
  const ACC sb = g.conjB ? ACC(-1) : ACC(1);
  const bool akf = g.a_kfast, bkf = g.b_kfast;

  // this thread's load slots: element u of a k-tile is (row ra(u), k ka(u)) of A, (k kb(u), col cb(u)) of B
  auto ra = [&](int u) { return akf ? tid / BK + (NT / BK) * u : tid % BM; };
  auto ka = [&](int u) { return akf ? tid % BK : tid / BM + (NT / BM) * u; };
  auto cb = [&](int u) { return bkf ? tid / BK + (NT / BK) * u : tid % BN; };
  auto kb = [&](int u) { return bkf ? tid % BK : tid / BN + (NT / BN) * u; };
  int offm[EA], offn[EB];
#pragma unroll
  for (int u = 0; u < EA; ++u) {
    const int m = m0 + ra(u);
    offm[u] = m < M ? g.offAm[m] : -1;
  }
#pragma unroll
  for (int u = 0; u < EB; ++u) {
    const int n = n0 + cb(u);
    offn[u] = n < N ? g.offBn[n] : -1;
  }
  CA ra_v[EA];
  CB rb_v[EB];
  // the k offsets of a k-tile are read one tile ahead of its data (fetch_k), so that a data fetch
  // does not wait for its table lookup; -1 marks k >= K
  int koA[EA], koB[EB];
  auto fetch_k = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int k = k0 + ka(u);
      koA[u] = k < K ? g.offAk[k] : -1;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int k = k0 + kb(u);
      koB[u] = k < K ? g.offBk[k] : -1;
    }
  };
  auto fetch = [&]() {
#pragma unroll
    for (int u = 0; u < EA; ++u)
      ra_v[u] = (offm[u] >= 0 && koA[u] >= 0) ? A[(int64_t)offm[u] + koA[u]] : CA{0, 0};
#pragma unroll
    for (int u = 0; u < EB; ++u)
      rb_v[u] = (offn[u] >= 0 && koB[u] >= 0) ? B[(int64_t)koB[u] + offn[u]] : CB{0, 0};
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      sAr[buf][ka(u)][ra(u)] = ACC(ra_v[u].x);
      sAi[buf][ka(u)][ra(u)] = sa * ACC(ra_v[u].y);
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      sBr[buf][kb(u)][cb(u)] = ACC(rb_v[u].x);
      sBi[buf][kb(u)][cb(u)] = sb * ACC(rb_v[u].y);
    }
  };

  V4 accr[MB][NB], acci[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      accr[i][j] = V4{0, 0, 0, 0};
      acci[i][j] = V4{0, 0, 0, 0};
    }

  fetch_k(kbeg);
  fetch();
  stash(0);
  fetch_k(kbeg + BK);
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) {
      fetch();                  // tile k0 + BK, offsets read during the previous tile
      fetch_k(k0 + 2 * BK);     // offsets of the tile after it
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      ACC ar[MB], ai[MB], br[NB], bi[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        ar[i] = sAr[buf][kr][wr * WM + i * 16 + (lane & 15)];
        ai[i] = sAi[buf][kr][wr * WM + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        br[j] = sBr[buf][kr][wc * WN + j * 16 + (lane & 15)];
        bi[j] = sBi[buf][kr][wc * WN + j * 16 + (lane & 15)];
      }
      // the two products into each accumulator are issued a full sweep apart, so dependent MFMAs
      // never follow each other
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accr[i][j] = mfma16(ar[i], br[j], accr[i][j]);
          acci[i][j] = mfma16(ar[i], bi[j], acci[i][j]);
        }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accr[i][j] = mfma16(-ai[i], bi[j], accr[i][j]);
          acci[i][j] = mfma16(ai[i], br[j], acci[i][j]);
        }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // output rows of a 16x16 block: FP32 MFMA lane l, register r -> row 4*(l/16) + r; FP64 MFMA ->
  // row l/16 + 4*r (column l%16 in both)
  auto row_of = [&](int r) { return F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r; };
  if (g.ksplit > 1) {
    // raw chunk sums, row-major M x N per (instance, chunk)
    using CP = typename Cplx<ACC>::type;
    CP* __restrict__ P = reinterpret_cast<CP*>(inst_ptr(g.part, g.bsPart, bz)) + (int64_t)kz * M * N;
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int n = n0 + wc * WN + j * 16 + (lane & 15);
        if (n >= N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wr * WM + i * 16 + row_of(r);
          if (m < M) P[(int64_t)m * N + n] = CP{accr[i][j][r], acci[i][j][r]};
        }
      }
    return;
  }
  double alpha = g.alpha;
  if (g.alpha_dev) alpha *= inst_ptr(g.alpha_dev, g.bsAlpha, bz)[0];
  if (g.alpha_dev2) alpha *= inst_ptr(g.alpha_dev2, g.bsAlpha2, bz)[0];
  CC* __restrict__ C = reinterpret_cast<CC*>(inst_ptr(g.C, g.bsC, bz));
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wc * WN + j * 16 + (lane & 15);
      if (n >= N) continue;
      const int32_t cn = g.offCn[n];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wr * WM + i * 16 + row_of(r);
        if (m < M && (!g.herm || m >= n)) {
          CC out;
          out.x = TC(double(accr[i][j][r]) * alpha);
          out.y = TC(double(acci[i][j][r]) * alpha);
          C[(int64_t)g.offCm[m] + cn] = out;
          if (g.herm && m > n) {
            out.y = -out.y;
            C[(int64_t)g.offCm[n] + g.offCn[m]] = out;
          }
        }
      }
    }
}

// Entry points of the pipelined kernel. With FP32 operands and accumulation the register budget is
// capped at four waves per SIMD (128 registers, no spills), so that a launch of up to 1024 64 x 64
// tiles runs in one round on the 256 compute units; the other instantiations keep the compiler's
// own budget (the cap would spill their staging registers).
template <typename TA, typename TB, typename TC, typename ACC, int BM, int BN>
__global__ __launch_bounds__(256) void k_cgemm_pipe(GemmArgs g) {
  cgemm_pipe_body<TA, TB, TC, ACC, BM, BN>(g);
}
template <typename TA, typename TB, typename TC, typename ACC, int BM, int BN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_cgemm_pipe4(GemmArgs g) {
  cgemm_pipe_body<TA, TB, TC, ACC, BM, BN>(g);
}
// 128 x 128 tiles on eight waves (2 x 4, each 64 x 32), k-tiles of 8: a quarter of the 64 x 64
// tile's operand traffic per product, for the largest FP32 contractions
template <typename TA, typename TB, typename TC, typename ACC>
__global__ __launch_bounds__(512) void k_cgemm_pipe128(GemmArgs g) {
  cgemm_pipe_body<TA, TB, TC, ACC, 128, 128, 2, 4>(g);
}

// Tile choice by shape (measured on MI355X): with FP32 accumulation the pipelined 64x64 kernel
// whenever there are at least 64 such output tiles (split along K below 512 tiles, see
// gemm_pick_ksplit); otherwise, and for FP64 accumulation, the table-driven 32x32 kernel, whose many
// small workgroups hide latency best.
int gemm_pick_tile(int M, int N, int K, int batch, bool fp64_acc) {
  const int64_t t64 = (int64_t)((M + 63) / 64) * ((N + 63) / 64) * batch;
  if (!fp64_acc && M >= 64 && N >= 64 && K >= 16 &&
      (t64 >= 512 || (t64 >= 64 && K >= 512)))
    return GEMM_PIPE64;
  return GEMM_TILE32;
}

// Split-K for launches with fewer than 512 output tiles and a reduction of at least 128: chunks
// until there are about 1024 workgroups, at most max(K / 256, min(8, K / 16)) of them (up to 64).
// On MI355X the autotuner picks 8 chunks for the small Grams and projections of the 64-site
// workload (e.g. 64 x 64 x 128 FP64: 17 -> 9.4 us; 128 x 128 x 512: 33 -> 15 us).
int gemm_pick_ksplit(int M, int N, int K, int batch, int tile) {
  if (K < 128) return 1;
  const int bm = tile == GEMM_TILE32 ? 32 : 64;
  const int64_t tiles = (int64_t)((M + bm - 1) / bm) * ((N + bm - 1) / bm) * batch;
  if (tiles >= 512) return 1;
  int64_t ks = (1024 + tiles - 1) / tiles;
  const int64_t kmax = std::max<int64_t>(K / 256, std::min<int64_t>(8, K / 16));
  if (ks > kmax) ks = kmax;
  if (ks > 64) ks = 64;
  return ks < 2 ? 1 : (int)ks;
}

template <typename TA, typename TB, typename TC, typename ACC>
static hipError_t launch_t(const GemmArgs& a0, int tile, hipStream_t s) {
  if (a0.M <= 0 || a0.N <= 0 || a0.batch <= 0) return hipSuccess;
  if (tile == GEMM_AUTO) tile = gemm_pick_tile(a0.M, a0.N, a0.K, a0.batch, sizeof(ACC) == 8);
  if (tile != GEMM_TILE32 && tile != GEMM_TILE64 && tile != GEMM_PIPE64 && tile != GEMM_PIPE128)
    return hipErrorInvalidValue;
  // the pipelined kernels: offset tables, no accumulation into C; 128 x 128 tiles with FP32
  // accumulation only
  if (tile == GEMM_PIPE128 && sizeof(ACC) == 8) tile = GEMM_PIPE64;
  if ((tile == GEMM_PIPE64 || tile == GEMM_PIPE128) && (!a0.offAm || a0.accum)) tile = GEMM_TILE64;
  if (a0.herm && (a0.M != a0.N || a0.accum)) return hipErrorInvalidValue;
  const bool split = a0.ksplit > 1;
  if (split && (tile == GEMM_TILE64 || !a0.part || a0.kchunk % 16 != 0 ||
                (int64_t)a0.kchunk * a0.ksplit < a0.K))
    return hipErrorInvalidValue;
  if ((int64_t)a0.batch * a0.ksplit > 65535) return hipErrorInvalidValue;
  const int BMt = tile == GEMM_TILE32 ? 32 : tile == GEMM_PIPE128 ? 128 : 64;
  const int max_rows = 65535 * BMt;   // grid y limit per launch
  if (split && a0.M > max_rows) return hipErrorInvalidValue;
  for (int mb = 0; mb < a0.M; mb += max_rows) {
    GemmArgs a = a0;
    a.mbase = mb;
    const int rows = a0.M - mb < max_rows ? a0.M - mb : max_rows;
    const dim3 grid((a.N + BMt - 1) / BMt, (rows + BMt - 1) / BMt, a.batch * a.ksplit);
    if (tile == GEMM_PIPE128) {
      if constexpr (sizeof(ACC) == 4)
        hipLaunchKernelGGL((k_cgemm_pipe128<TA, TB, TC, ACC>), grid, dim3(512), 0, s, a);
    } else if (tile == GEMM_PIPE64) {
      if constexpr (sizeof(TA) == 4 && sizeof(TB) == 4 && sizeof(ACC) == 4)
        hipLaunchKernelGGL((k_cgemm_pipe4<TA, TB, TC, ACC, 64, 64>), grid, dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((k_cgemm_pipe<TA, TB, TC, ACC, 64, 64>), grid, dim3(256), 0, s, a);
    } else if (tile == GEMM_TILE64)
      hipLaunchKernelGGL((k_cgemm<TA, TB, TC, ACC, 64, 64>), grid, dim3(256), 0, s, a);
    else if (a.offAm && !a.accum)
      // 32 x 32 tiles from offset tables: the pipelined body (same products in the same order,
      // the next k-tile fetched while the current one is consumed)
      hipLaunchKernelGGL((k_cgemm_pipe<TA, TB, TC, ACC, 32, 32>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_cgemm<TA, TB, TC, ACC, 32, 32>), grid, dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (split) {
    const int64_t mn = (int64_t)a0.M * a0.N;
    hipLaunchKernelGGL((k_splitk_reduce<TC, ACC>), dim3((unsigned)((mn + 255) / 256), a0.batch),
                       dim3(256), 0, s, a0);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <typename ACC>
static hipError_t launch_acc(const GemmArgs& a, DType ta, DType tb, DType tc, int tile,
                             hipStream_t s) {
  const int code = (ta == DT_C128 ? 4 : 0) | (tb == DT_C128 ? 2 : 0) | (tc == DT_C128 ? 1 : 0);
  switch (code) {
    case 0: return launch_t<float, float, float, ACC>(a, tile, s);
    case 1: return launch_t<float, float, double, ACC>(a, tile, s);
    case 2: return launch_t<float, double, float, ACC>(a, tile, s);
    case 3: return launch_t<float, double, double, ACC>(a, tile, s);
    case 4: return launch_t<double, float, float, ACC>(a, tile, s);
    case 5: return launch_t<double, float, double, ACC>(a, tile, s);
    case 6: return launch_t<double, double, float, ACC>(a, tile, s);
    default: return launch_t<double, double, double, ACC>(a, tile, s);
  }
}

hipError_t launch_gemm(const GemmArgs& a, DType ta, DType tb, DType tc, DType acc, int tile,
                       hipStream_t s) {
  if (acc == DT_C128) return launch_acc<double>(a, ta, tb, tc, tile, s);
  return launch_acc<float>(a, ta, tb, tc, tile, s);
}

}  // namespace cbc
