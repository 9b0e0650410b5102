// Complex128 strided-batched products on the gfx950 FP64 matrix cores.
//
// One workgroup computes a BM x BN tile of D for one (group, batch entry).
// Operand tiles are staged through LDS in a k-major layout (As[k][m],
// Bs[k][n]) so that the 16 lanes feeding one MFMA row read 256 contiguous
// bytes.  Complex numbers stay interleaved (re, im): each lane reads one
// 16-byte complex per fragment and the complex product is four real
// v_mfma_f64_16x16x4_f64:
//     Cr += ar*br - ai*bi,   Ci += ar*bi + ai*br.
// MFMA operand layout (measured on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; accumulator register j of lane l is D[4j + l/16][l%16].
// Conjugate-transposed operands are read with the transposed global index
// and conjugated on the way into LDS.
#include "qtx_internal.h"

// Row held by accumulator register r of lane group lk (= lane / 16) for
// v_mfma_f32_16x16x4_f32.
#ifndef QTX_F32_ROW
#define QTX_F32_ROW(r, lk) (4 * (lk) + (r))
#endif

namespace qtx {
namespace {

// Arithmetic of the matrix-core product.  Operands always live in HBM as
// complex128; the FP32 variant rounds them to complex64 on the way into LDS
// and accumulates in FP32, while the epilogue (alpha, beta, C) stays FP64.
struct MathF64 {
  typedef double2 lds_t;
  typedef d4v acc_t;
  typedef double real_t;
  static __device__ __forceinline__ lds_t cvt(double2 v) { return v; }
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register r of lane group lk holds row 4r + lk
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
};
struct MathF32 {
  typedef float2 lds_t;
  typedef f4v acc_t;
  typedef float real_t;
  static __device__ __forceinline__ lds_t cvt(double2 v) {
    return make_float2((float)v.x, (float)v.y);
  }
  static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return QTX_F32_ROW(r, lk); }
};

template <int OPA, int OPB, int BM, int BN, int BK, int WGM, int WGN>
struct ZTile {
  static constexpr int kThreads = 64 * WGM * WGN;
  static constexpr int kWM = BM / WGM;       // rows per wave
  static constexpr int kWN = BN / WGN;       // columns per wave
  static constexpr int kTM = kWM / 16;       // MFMA tiles per wave (rows)
  static constexpr int kTN = kWN / 16;
  static constexpr int kPad = 1;
  static constexpr int kLdA = BM + kPad;
  static constexpr int kLdB = BN + kPad;
  static constexpr int kALoads = BM * BK / kThreads;
  static constexpr int kBLoads = BN * BK / kThreads;
  static_assert(BM * BK % kThreads == 0 && BN * BK % kThreads == 0, "tile");
  static_assert(kWM % 16 == 0 && kWN % 16 == 0 && BK % 4 == 0, "tile");
};

template <class P, int OPA, int OPB, int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN)
void zgemm_kernel(GemmArgs args) {
  using T = ZTile<OPA, OPB, BM, BN, BK, WGM, WGN>;
  typedef typename P::lds_t L;
  typedef typename P::acc_t Acc;
  typedef typename P::real_t R;
  __shared__ L As[2][BK][T::kLdA];
  __shared__ L Bs[2][BK][T::kLdB];

  const GemmGroup& g = args.g[blockIdx.z];
  const int M = args.M, N = args.N, K = args.K;
  const int tilesN = (N + BN - 1) / BN;
  const int m0 = (blockIdx.x / tilesN) * BM;
  const int n0 = (blockIdx.x % tilesN) * BN;
  const int nb2 = args.batch2 > 0 ? args.batch2 : 1;
  const long long e = blockIdx.y / nb2;
  const long long i2 = blockIdx.y % nb2;
  const double2* __restrict__ A = (const double2*)g.A + e * g.sA + i2 * g.tA;
  const double2* __restrict__ B = (const double2*)g.B + e * g.sB + i2 * g.tB;
  const long long lda = args.lda, ldb = args.ldb;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  double2 ra[T::kALoads], rb[T::kBLoads];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int r = 0; r < T::kALoads; ++r) {
      int q = tid + r * T::kThreads;
      int m, k;
      if (OPA == 0) { m = q / BK; k = q % BK; } else { k = q / BM; m = q % BM; }
      int gm = m0 + m, gk = k0 + k;
      double2 v = make_double2(0.0, 0.0);
      if (gm < M && gk < K)
        v = (OPA == 0) ? A[(long long)gm * lda + gk] : A[(long long)gk * lda + gm];
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < T::kBLoads; ++r) {
      int q = tid + r * T::kThreads;
      int n, k;
      if (OPB == 0) { k = q / BN; n = q % BN; } else { n = q / BK; k = q % BK; }
      int gn = n0 + n, gk = k0 + k;
      double2 v = make_double2(0.0, 0.0);
      if (gn < N && gk < K)
        v = (OPB == 0) ? B[(long long)gk * ldb + gn] : B[(long long)gn * ldb + gk];
      rb[r] = v;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int r = 0; r < T::kALoads; ++r) {
      int q = tid + r * T::kThreads;
      int m, k;
      if (OPA == 0) { m = q / BK; k = q % BK; } else { k = q / BM; m = q % BM; }
      L v = P::cvt(ra[r]);
      if (OPA == 1) v.y = -v.y;
      As[buf][k][m] = v;
    }
#pragma unroll
    for (int r = 0; r < T::kBLoads; ++r) {
      int q = tid + r * T::kThreads;
      int n, k;
      if (OPB == 0) { k = q / BN; n = q % BN; } else { n = q / BK; k = q % BK; }
      L v = P::cvt(rb[r]);
      if (OPB == 1) v.y = -v.y;
      Bs[buf][k][n] = v;
    }
  };

  Acc accR[T::kTM][T::kTN], accI[T::kTM][T::kTN];
#pragma unroll
  for (int i = 0; i < T::kTM; ++i)
#pragma unroll
    for (int j = 0; j < T::kTN; ++j) {
      accR[i][j] = Acc{0, 0, 0, 0};
      accI[i][j] = Acc{0, 0, 0, 0};
    }

  const int nk = (K + BK - 1) / BK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  const int lrow = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kidx = kk * 4 + lk;
      L a[T::kTM], b[T::kTN];
#pragma unroll
      for (int i = 0; i < T::kTM; ++i) a[i] = As[buf][kidx][wm * T::kWM + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < T::kTN; ++j) b[j] = Bs[buf][kidx][wn * T::kWN + j * 16 + lrow];
#pragma unroll
      for (int i = 0; i < T::kTM; ++i) {
        const R nai = -a[i].y;
#pragma unroll
        for (int j = 0; j < T::kTN; ++j) {
          accR[i][j] = P::mfma(a[i].x, b[j].x, accR[i][j]);
          accI[i][j] = P::mfma(a[i].x, b[j].y, accI[i][j]);
          accR[i][j] = P::mfma(nai, b[j].y, accR[i][j]);
          accI[i][j] = P::mfma(a[i].y, b[j].x, accI[i][j]);
        }
      }
    }
    if (kt + 1 < nk) store_tiles(buf ^ 1);
    __syncthreads();
  }

  // epilogue: D = alpha * acc + beta * C
  double2* __restrict__ D = (double2*)g.D + e * g.sD + i2 * g.tD;
  const double2* __restrict__ C = g.C ? (const double2*)g.C + e * g.sC + i2 * g.tC : nullptr;
  const bool useC = (g.beta.re != 0.0 || g.beta.im != 0.0) && C != nullptr;
  const long long ldc = args.ldc, ldd = args.ldd;
#pragma unroll
  for (int i = 0; i < T::kTM; ++i)
#pragma unroll
    for (int j = 0; j < T::kTN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * T::kWM + i * 16 + P::row(r, lk);
        const int gn = n0 + wn * T::kWN + j * 16 + lrow;
        if (gm < M && gn < N) {
          double2 v = cscale(g.alpha, make_double2((double)accR[i][j][r], (double)accI[i][j][r]));
          if (useC) v = cadd(v, cscale(g.beta, C[(long long)gm * ldc + gn]));
          D[(long long)gm * ldd + gn] = v;
        }
      }
}

template <class P, int OPA, int OPB>
hipError_t launch_t(const GemmArgs& a, hipStream_t s) {
  constexpr int BM = 64, BN = 64, BK = 16, WGM = 2, WGN = 2;
  const int nb2 = a.batch2 > 0 ? a.batch2 : 1;
  dim3 grid(((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN), a.batch * nb2, a.ngroups);
  hipLaunchKernelGGL((zgemm_kernel<P, OPA, OPB, BM, BN, BK, WGM, WGN>), grid,
                     dim3(64 * WGM * WGN), 0, s, a);
  return hipGetLastError();
}

template <class P>
hipError_t dispatch(char opa, char opb, const GemmArgs& a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0 || a.ngroups <= 0) return hipSuccess;
  const int oa = (opa == 'C'), ob = (opb == 'C');
  if (oa == 0 && ob == 0) return launch_t<P, 0, 0>(a, s);
  if (oa == 0 && ob == 1) return launch_t<P, 0, 1>(a, s);
  if (oa == 1 && ob == 0) return launch_t<P, 1, 0>(a, s);
  return launch_t<P, 1, 1>(a, s);
}

}  // namespace

hipError_t launch_zgemm(char opa, char opb, const GemmArgs& a, hipStream_t s) {
  return dispatch<MathF64>(opa, opb, a, s);
}

hipError_t launch_cgemm(char opa, char opb, const GemmArgs& a, hipStream_t s) {
  return dispatch<MathF32>(opa, opb, a, s);
}

}  // namespace qtx
