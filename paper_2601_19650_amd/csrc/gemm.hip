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
  const int M = g.M, N = g.N, K = g.K;
  const int bz = blockIdx.z;
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

  for (int k0 = 0; k0 < K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int r, kk;
      if (g.a_kfast) { kk = e % BK; r = e / BK; } else { r = e % BM; kk = e / BM; }
      const int m = m0 + r, k = k0 + kk;
      ACC re = 0, im = 0;
      if (m < M && k < K) {
        const CA v = A[(int64_t)g.offAm[m] + g.offAk[k]];
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
        const CB v = B[(int64_t)g.offBk[k] + g.offBn[n]];
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
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accr[i][j] = mfma16(ar[i], br[j], accr[i][j]);
          accr[i][j] = mfma16(-ai[i], bi[j], accr[i][j]);
          acci[i][j] = mfma16(ar[i], bi[j], acci[i][j]);
          acci[i][j] = mfma16(ai[i], br[j], acci[i][j]);
        }
    }
    __syncthreads();
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
        // output rows of a 16x16 block: FP32 MFMA lane l, register r -> row 4*(l/16) + r;
        // FP64 MFMA -> row l/16 + 4*r (column l%16 in both)
        const int rb = sizeof(ACC) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int m = m0 + wr * WM + i * 16 + rb;
        if (m < M) {
          CC out;
          out.x = TC(double(accr[i][j][r]) * alpha);
          out.y = TC(double(acci[i][j][r]) * alpha);
          C[(int64_t)g.offCm[m] + cn] = out;
        }
      }
    }
}

template <typename TA, typename TB, typename TC, typename ACC>
static hipError_t launch_t(const GemmArgs& a0, int tile, hipStream_t s) {
  if (a0.M <= 0 || a0.N <= 0 || a0.batch <= 0) return hipSuccess;
  const int BMt = tile == 1 ? 64 : 32;
  const int max_rows = 65535 * BMt;   // grid y limit per launch
  for (int mb = 0; mb < a0.M; mb += max_rows) {
    GemmArgs a = a0;
    a.mbase = mb;
    const int rows = a0.M - mb < max_rows ? a0.M - mb : max_rows;
    if (tile == 1) {
      dim3 grid((a.N + 63) / 64, (rows + 63) / 64, a.batch);
      hipLaunchKernelGGL((k_cgemm<TA, TB, TC, ACC, 64, 64>), grid, dim3(256), 0, s, a);
    } else {
      dim3 grid((a.N + 31) / 32, (rows + 31) / 32, a.batch);
      hipLaunchKernelGGL((k_cgemm<TA, TB, TC, ACC, 32, 32>), grid, dim3(256), 0, s, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
