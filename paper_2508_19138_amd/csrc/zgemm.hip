// Complex strided-batched products on the gfx950 matrix cores.
//
// A workgroup computes one BM x BN tile of D for one matrix of one
// descriptor.  Operand tiles are staged through LDS in the layout in which
// they are read from HBM, double buffered; whole tiles go from HBM straight
// into LDS without passing through registers (see zgemm_kernel).  Complex
// numbers stay interleaved (re, im): each lane reads one complex per
// fragment.  FP64 products take three real MFMAs per complex product (the
// 3M form, see zgemm_kernel); FP32 products four,
//     Cr += ar*br - ai*bi,   Ci += ar*bi + ai*br.
// MFMA operand layout (measured on gfx950, both 16x16x4 f64 and f32): lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register r of lane l
// holds D[4r + l/16][l%16] for f64 and D[4(l/16) + r][l%16] for f32.
// Conjugate-transposed operands are read with the transposed global index
// and conjugated as their fragments are read from LDS.  Workgroup ids are
// remapped so that the tiles of one matrix land on the same XCD (shared L2).
#include "qtx_internal.h"

namespace qtx {
namespace {

// Operands live in HBM (and LDS) as complex128; the FP32 variant rounds them
// to complex64 as the fragments are read and accumulates in FP32, while the
// epilogue (alpha, beta, C) stays FP64.
struct MathF64 {
  typedef double2 lds_t;
  typedef d4v acc_t;
  typedef double real_t;
  static __device__ __forceinline__ lds_t cvt(double2 v) { return v; }
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
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
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
};

template <int BM_, int BN_, int BK_, int WGM_, int WGN_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
  static constexpr int kThreads = 64 * WGM * WGN;
  static constexpr int kWM = BM / WGM;
  static constexpr int kWN = BN / WGN;
  static constexpr int kTM = kWM / 16;
  static constexpr int kTN = kWN / 16;
  static constexpr int kALoads = BM * BK / kThreads;
  static constexpr int kBLoads = BN * BK / kThreads;
  static_assert(BM * BK % kThreads == 0 && BN * BK % kThreads == 0, "tile");
  static_assert(kWM % 16 == 0 && kWN % 16 == 0 && BK % 4 == 0, "tile");
};

// FP64 products use the 3M form (three accumulator sets, so 32 x 32 per
// wave), the inverse's thin update products included (measured 4-7% faster
// inverses at 128 matrices than with four products); FP32 products the
// four-product form (FP32's 3M form measured 4x less accurate in the
// partitioned solve).
typedef Cfg<64, 64, 8, 2, 2> Cfg0;      // general, 3M: 32 x 32 per wave, three waves per SIMD
typedef Cfg<64, 64, 8, 2, 2> Cfg0w;     // general, four products
typedef Cfg<128, 64, 8, 4, 2> Cfg1;    // large blocks, 3M: eight waves of 32 x 32
typedef Cfg<128, 64, 8, 2, 2> Cfg1w;   // large blocks, four products: 64 x 32 per wave
typedef Cfg<32, 32, 16, 2, 2> Cfg2;     // small blocks
typedef Cfg<32, 32, 16, 2, 2> CfgU;     // the inverse's update products
static_assert(Cfg1w::BM == Cfg1::BM && Cfg1w::BN == Cfg1::BN, "one tile shape per configuration");
static_assert(Cfg0w::BM == Cfg0::BM && Cfg0w::BN == Cfg0::BN, "one tile shape per configuration");
static_assert(CfgU::BM == kInvUpdTile && CfgU::BN == kInvUpdTile, "update tile");
static_assert(Cfg0::BM == kMegaTile && Cfg0::BN == kMegaTile, "mega tile");

__device__ __forceinline__ int xcd_remap(int w, int G) {
  constexpr int kXcd = 8;
  const int per = G / kXcd;
  if (w < per * kXcd) return (w % kXcd) * per + (w / kXcd);
  return w;
}

// Direct layout of an operand tile (the slot of each element in LDS).
// A k-major tile (BK rows k of BW consecutive elements) is stored as read.
// A row-major tile (BW rows w of BK consecutive k) permutes the k slots of
// row w by XOR with (w / rows per 256 bytes) % BK, so that the 16 lanes that
// read 16 consecutive rows at one k hit distinct banks; the lanes that fill
// a row still read its contiguous segment of HBM.  swz_slot gives the slot
// of (w, k), slot_elem the element of slot s (the XOR is its own inverse).
template <int BK>
__device__ __forceinline__ int swz_slot(int w, int k) {
  static_assert((BK & (BK - 1)) == 0, "the XOR permutation needs a power-of-two BK");
  constexpr int kRPB = 16 * BK >= 256 ? 1 : 256 / (16 * BK);
  return w * BK + (k ^ ((w / kRPB) % BK));
}
template <int BK, int BW, int TRANS>
__device__ __forceinline__ void slot_elem(int s, int& w, int& k) {
  if (TRANS) {
    constexpr int kRPB = 16 * BK >= 256 ? 1 : 256 / (16 * BK);
    w = s / BK;
    k = (s % BK) ^ ((w / kRPB) % BK);
  } else {
    k = s / BW;
    w = s % BW;
  }
}

// One complex from HBM into LDS without registers (global_load_lds_dwordx4):
// the lane's 16 bytes land at lds_wave + 16 * (lane index), lds_wave being
// the same for the whole wave.  Completion is counted by vmcnt.
__device__ __forceinline__ void lds_dma16(const double2* src, double2* lds_wave) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)lds_wave, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// CM = 4: each complex product is four real products,
//     Cr += ar br - ai bi,  Ci += ar bi + ai br;
// CM = 3: three (the 3M form), accumulated separately and combined in the
// epilogue,
//     T1 += ar br,  T2 += ai bi,  T3 += (ar + ai)(br + bi),
//     Cr = T1 - T2,  Ci = T3 - T1 - T2.
// The 3M form does three quarters of the matrix-core work.  Its real part
// is the conventional one; its imaginary part is bounded by a small multiple
// of u (|Ar| + |Ai|)(|Br| + |Bi|) instead of u (|Ar||Bi| + |Ai||Br|), the
// same order for operands whose real and imaginary parts are of similar
// size (the stability analysis of the three-multiplication method).  Every
// tile configuration uses the same form and the same k order, so the tile
// still changes no bit of a result.
// TAG only separates kernel symbols (1 = rank-kPanel and rank-kSuper
// updates of the inverse, 2 = its rank-kMega updates) so that profilers
// report the uses apart.
template <class P, class T, int OPA, int OPB, int TAG, int CM>
__global__ __launch_bounds__(T::kThreads)
void zgemm_kernel(FlatLaunch L) {
  typedef typename P::lds_t Lt;
  typedef typename P::acc_t Acc;
  typedef typename P::real_t R;
  constexpr int BM = T::BM, BN = T::BN, BK = T::BK, WGN = T::WGN;
  // Each operand tile keeps the layout in which it arrives from HBM: A
  // (row = m) and B^dagger (row = n) row-major, A^dagger and B (row = k)
  // k-major.
  // Whole tiles go from HBM straight into LDS, one complex128 per lane,
  // without passing through registers (see slot_elem); the layout is
  // unpadded and the row-major tiles permute the k slots of each row.  The
  // adjoint operands are conjugated, and FP32 operands rounded to complex64,
  // as their fragments are read.  Tiles that cross the edge of a matrix load
  // through registers into the same layout, with zeros outside.
  // The two buffers of each operand are separate arrays: the compiler can
  // then tell a read of one buffer from the direct loads into the other and
  // does not make the read wait for them.
  __shared__ double2 As0[BM * BK], As1[BM * BK];
  __shared__ double2 Bs0[BN * BK], Bs1[BN * BK];
  auto ia = [](int k, int m) { return OPA == 0 ? swz_slot<BK>(m, k) : k * BM + m; };
  auto ib = [](int k, int n) { return OPB == 1 ? swz_slot<BK>(n, k) : k * BN + n; };

  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int di = find_desc(L.prefix, L.nd, w);
  const GemmDesc& g = ((const GemmDesc*)L.desc)[di];
  const int local = w - L.prefix[di];
  const int mat = local / g.tiles;
  const int tile = local % g.tiles;
  const int M = g.M, N = g.N, K = g.K;
  const int tilesN = (N + BN - 1) / BN;
  const int m0 = (tile / tilesN) * BM;
  const int n0 = (tile % tilesN) * BN;
  const int nb2 = g.batch2 > 0 ? g.batch2 : 1;
  const long long e = mat / nb2;
  const long long i2 = mat % nb2;
  const double2* __restrict__ A = (const double2*)g.A + e * g.sA + i2 * g.tA;
  const double2* __restrict__ B = (const double2*)g.B + e * g.sB + i2 * g.tB;
  const long long lda = g.lda, ldb = g.ldb;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  double2 ra[T::kALoads], rb[T::kBLoads];

  // whole tile inside the matrices: loads need no bounds checks
  const bool full = (m0 + BM <= M) && (n0 + BN <= N) && (K % BK == 0);
  // tiles that cross an edge: through registers, zeros outside the matrices
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int r = 0; r < T::kALoads; ++r) {
      const int q = tid + r * T::kThreads;
      int m, k;
      slot_elem<BK, BM, OPA == 0>(q, m, k);
      const int gm = m0 + m, gk = k0 + k;
      double2 v = make_double2(0.0, 0.0);
      if (gm < M && gk < K)
        v = (OPA == 0) ? A[(long long)gm * lda + gk] : A[(long long)gk * lda + gm];
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < T::kBLoads; ++r) {
      const int q = tid + r * T::kThreads;
      int n, k;
      slot_elem<BK, BN, OPB == 1>(q, n, k);
      const int gn = n0 + n, gk = k0 + k;
      double2 v = make_double2(0.0, 0.0);
      if (gn < N && gk < K)
        v = (OPB == 0) ? B[(long long)gk * ldb + gn] : B[(long long)gn * ldb + gk];
      rb[r] = v;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int r = 0; r < T::kALoads; ++r) (buf ? As1 : As0)[tid + r * T::kThreads] = ra[r];
#pragma unroll
    for (int r = 0; r < T::kBLoads; ++r) (buf ? Bs1 : Bs0)[tid + r * T::kThreads] = rb[r];
  };

  constexpr int kS = CM == 3 ? 1 : 0;          // third accumulator set (3M)
  Acc accR[T::kTM][T::kTN], accI[T::kTM][T::kTN];
  Acc accS[kS ? T::kTM : 1][kS ? T::kTN : 1];
#pragma unroll
  for (int i = 0; i < T::kTM; ++i)
#pragma unroll
    for (int j = 0; j < T::kTN; ++j) {
      accR[i][j] = Acc{0, 0, 0, 0};
      accI[i][j] = Acc{0, 0, 0, 0};
      if (kS) accS[kS ? i : 0][kS ? j : 0] = Acc{0, 0, 0, 0};
    }

  // the inverse's update products (K = 16 or 64) read C before the k loop,
  // so that its latency overlaps the operand loads and the products
  constexpr bool kPreC = (TAG == 1);
  double2 cpre[kPreC ? T::kTM : 1][kPreC ? T::kTN : 1][4];
  if (kPreC) {
    const double2* __restrict__ Cp = g.C ? (const double2*)g.C + e * g.sC + i2 * g.tC : nullptr;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < T::kTM; ++i)
#pragma unroll
      for (int j = 0; j < T::kTN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm * T::kWM + i * 16 + P::row(r, lq);
          const int gn = n0 + wn * T::kWN + j * 16 + lr;
          cpre[i][j][r] = (Cp && gm < M && gn < N) ? Cp[(long long)gm * g.ldc + gn]
                                                   : make_double2(0.0, 0.0);
        }
  }
  // whole tiles: every lane of a wave instruction reads one complex from
  // HBM into the next 16-byte slot after the wave's base in LDS
  auto dma_tiles = [&](int k0, double2* as, double2* bs) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < T::kALoads; ++r) {
      const int q = tid + r * T::kThreads;
      int m, k;
      slot_elem<BK, BM, OPA == 0>(q, m, k);
      const double2* src = (OPA == 0) ? A + ((long long)(m0 + m) * lda + k0 + k)
                                      : A + ((long long)(k0 + k) * lda + m0 + m);
      lds_dma16(src, as + r * T::kThreads + wave * 64);
    }
#pragma unroll
    for (int r = 0; r < T::kBLoads; ++r) {
      const int q = tid + r * T::kThreads;
      int n, k;
      slot_elem<BK, BN, OPB == 1>(q, n, k);
      const double2* src = (OPB == 0) ? B + ((long long)(k0 + k) * ldb + n0 + n)
                                      : B + ((long long)(n0 + n) * ldb + k0 + k);
      lds_dma16(src, bs + r * T::kThreads + wave * 64);
    }
  };
  const int lrow = lane & 15, lk = lane >> 4;
  auto compute = [&](const double2* as, const double2* bs) __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kidx = kk * 4 + lk;
      Lt a[T::kTM], b[T::kTN];
#pragma unroll
      for (int i = 0; i < T::kTM; ++i) {
        a[i] = P::cvt(as[ia(kidx, wm * T::kWM + i * 16 + lrow)]);
        if (OPA == 1) a[i].y = -a[i].y;
      }
#pragma unroll
      for (int j = 0; j < T::kTN; ++j) {
        b[j] = P::cvt(bs[ib(kidx, wn * T::kWN + j * 16 + lrow)]);
        if (OPB == 1) b[j].y = -b[j].y;
      }
      if (CM == 3) {
        R as[T::kTM], bs[T::kTN];
#pragma unroll
        for (int i = 0; i < T::kTM; ++i) as[i] = a[i].x + a[i].y;
#pragma unroll
        for (int j = 0; j < T::kTN; ++j) bs[j] = b[j].x + b[j].y;
#pragma unroll
        for (int i = 0; i < T::kTM; ++i)
#pragma unroll
          for (int j = 0; j < T::kTN; ++j) {
            accR[i][j] = P::mfma(a[i].x, b[j].x, accR[i][j]);
            accI[i][j] = P::mfma(a[i].y, b[j].y, accI[i][j]);
            accS[kS ? i : 0][kS ? j : 0] = P::mfma(as[i], bs[j], accS[kS ? i : 0][kS ? j : 0]);
          }
      } else {
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
    }
  };
  const int nk = (K + BK - 1) / BK;
  // separate loops: in the direct one nothing waits for the next tile's
  // loads before the products of this one
  if (full) {
    // two k tiles per trip, so that every access names its buffer statically
    dma_tiles(0, As0, Bs0);
    lds_dma_wait();
    __syncthreads();
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {           // tile kt is in buffer 0
      dma_tiles((kt + 1) * BK, As1, Bs1);
      compute(As0, Bs0);
      lds_dma_wait();
      __syncthreads();
      if (kt + 2 < nk) dma_tiles((kt + 2) * BK, As0, Bs0);
      compute(As1, Bs1);
      lds_dma_wait();
      __syncthreads();
    }
    if (kt < nk) compute(As0, Bs0);          // an odd last tile
  } else {
    load_tiles(0);
    store_tiles(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load_tiles((kt + 1) * BK);
      compute(buf ? As1 : As0, buf ? Bs1 : Bs0);
      if (kt + 1 < nk) store_tiles(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: D = alpha * acc + beta * C
  double2* __restrict__ D = (double2*)g.D + e * g.sD + i2 * g.tD;
  const double2* __restrict__ C = g.C ? (const double2*)g.C + e * g.sC + i2 * g.tC : nullptr;
  const bool useC = (g.beta.re != 0.0 || g.beta.im != 0.0) && C != nullptr;
  const zc alpha = g.alpha, beta = g.beta;
  const long long ldc = g.ldc, ldd = g.ldd;
  // assembled C (same order of terms as the elementwise assembly pass)
  const bool asmC = TAG == 0 && g.asm_ != 0;
  zc aco[3] = {}, aid = {};
  const double2* __restrict__ AX[3] = {nullptr, nullptr, nullptr};
  if (asmC) {
    const double Ee = g.E ? g.E[e] : 0.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      aco[t] = zc{g.xc[t].re + g.xd[t].re * Ee, g.xc[t].im + g.xd[t].im * Ee};
      AX[t] = g.X[t] ? (const double2*)g.X[t] + e * g.sX[t] : nullptr;
    }
    aid = zc{g.i0.re + g.i1.re * Ee, g.i0.im + g.i1.im * Ee};
  }
#pragma unroll
  for (int i = 0; i < T::kTM; ++i)
#pragma unroll
    for (int j = 0; j < T::kTN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * T::kWM + i * 16 + P::row(r, lk);
        const int gn = n0 + wn * T::kWN + j * 16 + lrow;
        if (gm < M && gn < N) {
          double re, im;
          if (CM == 3) {
            const double t1 = (double)accR[i][j][r], t2 = (double)accI[i][j][r];
            re = t1 - t2;
            im = (double)accS[kS ? i : 0][kS ? j : 0][r] - t1 - t2;
          } else {
            re = (double)accR[i][j][r];
            im = (double)accI[i][j][r];
          }
          double2 v = cscale(alpha, make_double2(re, im));
          if (useC) v = cadd(v, cscale(beta, kPreC ? cpre[i][j][r] : C[(long long)gm * ldc + gn]));
          if (asmC) {
            const long long q = (long long)gm * ldc + gn;
            double2 cv = gm == gn ? make_double2(aid.re, aid.im) : make_double2(0.0, 0.0);
#pragma unroll
            for (int t = 0; t < 3; ++t)
              if (AX[t]) cv = cadd(cv, cscale(aco[t], AX[t][q]));
            v = cadd(v, cv);
          }
          D[(long long)gm * ldd + gn] = v;
        }
      }
}

template <class P, class T, int CM>
hipError_t launch_ops(char opa, char opb, const FlatLaunch& l, hipStream_t s) {
  const int oa = (opa == 'C'), ob = (opb == 'C');
  dim3 grid(l.total), block(T::kThreads);
  if (oa == 0 && ob == 0) hipLaunchKernelGGL((zgemm_kernel<P, T, 0, 0, 0, CM>), grid, block, 0, s, l);
  else if (oa == 0 && ob == 1) hipLaunchKernelGGL((zgemm_kernel<P, T, 0, 1, 0, CM>), grid, block, 0, s, l);
  else if (oa == 1 && ob == 0) hipLaunchKernelGGL((zgemm_kernel<P, T, 1, 0, 0, CM>), grid, block, 0, s, l);
  else hipLaunchKernelGGL((zgemm_kernel<P, T, 1, 1, 0, CM>), grid, block, 0, s, l);
  return hipGetLastError();
}

hipError_t launch_f64(int cfg, char opa, char opb, const FlatLaunch& l, hipStream_t s) {
  switch (cfg) {
    case 1: return launch_ops<MathF64, Cfg1, 3>(opa, opb, l, s);
    case 2: return launch_ops<MathF64, Cfg2, 3>(opa, opb, l, s);
    default: return launch_ops<MathF64, Cfg0, 3>(opa, opb, l, s);
  }
}

hipError_t launch_f32(int cfg, char opa, char opb, const FlatLaunch& l, hipStream_t s) {
  switch (cfg) {
    case 1: return launch_ops<MathF32, Cfg1w, 4>(opa, opb, l, s);
    case 2: return launch_ops<MathF32, Cfg2, 4>(opa, opb, l, s);
    default: return launch_ops<MathF32, Cfg0w, 4>(opa, opb, l, s);
  }
}

}  // namespace

int gemm_tile_m(int cfg) {
  return cfg == kGemmInvUpdate ? CfgU::BM : cfg == 1 ? Cfg1::BM : cfg == 2 ? Cfg2::BM : Cfg0::BM;
}
int gemm_tile_n(int cfg) {
  return cfg == kGemmInvUpdate ? CfgU::BN : cfg == 1 ? Cfg1::BN : cfg == 2 ? Cfg2::BN : Cfg0::BN;
}
// kGemmMegaUpdate (and every other value) falls through to configuration 0
// the inverse's update products use the small tile

hipError_t launch_gemm(int cfg, bool fp32, char opa, char opb, const FlatLaunch& l,
                       hipStream_t s) {
  if (l.total <= 0 || l.nd <= 0) return hipSuccess;
  if (cfg == kGemmInvUpdate) {
    hipLaunchKernelGGL((zgemm_kernel<MathF64, CfgU, 0, 0, 1, 3>), dim3(l.total),
                       dim3(CfgU::kThreads), 0, s, l);
    return hipGetLastError();
  }
  if (cfg == kGemmMegaUpdate) {       // the inverse's rank-kMega updates (TAG 2)
    hipLaunchKernelGGL((zgemm_kernel<MathF64, Cfg0, 0, 0, 2, 3>), dim3(l.total),
                       dim3(Cfg0::kThreads), 0, s, l);
    return hipGetLastError();
  }
  return fp32 ? launch_f32(cfg, opa, opb, l, s) : launch_f64(cfg, opa, opb, l, s);
}

}  // namespace qtx
