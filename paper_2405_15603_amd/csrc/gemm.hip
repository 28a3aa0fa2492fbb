// Kronecker factors and the loss gradient on the 16x16 MFMA tiles of gfx950.
//
// gemm_tn_splitk forms sums of outer products over all slab rows (Eq. KFAC-PINN:
// A = sum Z~ Z~^T, B = sum g g^T; the gradient sum (r/N) g Z~^T).  The
// contraction runs over slab rows (K = N*S up to 3e5), so K is split across
// workgroups; each split writes a partial tile and reduce_splitk sums them in
// FP64 in a fixed order (deterministic).  Operands are row-major over slab rows,
// so tiles are transposed on their way into LDS.  Modes: FP64, FP32, BF16, and
// BF16x3 (FP32 slabs split into BF16 hi + lo; hi*hi + lo*hi + hi*lo).
#include "common.h"
#include "fwdlap.h"
#include "launch.h"

namespace kp {

template <typename TS> struct TileCfg;
template <> struct TileCfg<bf16> { static constexpr int BM = 128, BN = 128, BK = 32, PAD = 8; };
template <> struct TileCfg<float> { static constexpr int BM = 128, BN = 128, BK = 16, PAD = 4; };
template <> struct TileCfg<double> { static constexpr int BM = 64, BN = 64, BK = 16, PAD = 2; };

typedef uint4 v16;  // one 16-byte vector

template <typename TS>
__device__ __forceinline__ typename Mfma<TS>::frag load_frag(const TS* base, int lane, int ldk, int k0);

template <>
__device__ __forceinline__ bf16x8 load_frag<bf16>(const bf16* base, int lane, int ldk, int k0) {
  return *(const bf16x8*)(base + (lane & 15) * ldk + k0 + (lane >> 4) * 8);
}
template <>
__device__ __forceinline__ float load_frag<float>(const float* base, int lane, int ldk, int k0) {
  return base[(lane & 15) * ldk + k0 + (lane >> 4)];
}
template <>
__device__ __forceinline__ double load_frag<double>(const double* base, int lane, int ldk, int k0) {
  return base[(lane & 15) * ldk + k0 + (lane >> 4)];
}

// ---------------------------------------------------------------------------
// part[s] = sum_{k in split s} w(k) A[k]^T B[k]   (A: K x M, B: K x N, rows)
// ---------------------------------------------------------------------------
// Block -> (tile t, split): every split's tiles run on one XCD, so the slab rows
// of a split are fetched into that XCD's L2 once and read there by all of its
// tiles, which advance through the rows together.  Workgroups go to the XCDs
// round-robin by linear id: block b runs on XCD b % 8 as that XCD's (b / 8)-th
// block, and XCD x takes splits x, x + 8, ... in turn, all tiles of each.
// False for blocks past the last split (no rows).
__device__ __forceinline__ bool tn_block(int ntiles, int kchunk, int K, int& t, int& split,
                                         int b = blockIdx.x) {
  const int x = b & 7, i = b >> 3;
  split = x + 8 * (i / ntiles);
  t = i % ntiles;
  return (long)split * kchunk < K;
}

template <int MODE> struct TnOp;
template <> struct TnOp<M_F64> { typedef double TA; typedef double TL; static constexpr int NP = 1; };
template <> struct TnOp<M_F32> { typedef float TA; typedef float TL; static constexpr int NP = 1; };
template <> struct TnOp<M_BF16> { typedef bf16 TA; typedef bf16 TL; static constexpr int NP = 1; };
template <> struct TnOp<M_BF16X3> { typedef float TA; typedef bf16 TL; static constexpr int NP = 2; };

template <int MODE, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_gemm_tn(const typename TnOp<MODE>::TA* __restrict__ A,
                                                 long lda, const typename TnOp<MODE>::TA* __restrict__ B,
                                                 long ldb, int M, int N, int K,
                                                 const double* __restrict__ rw, int rmod, int sym,
                                                 int ntm, int ntn, int kchunk,
                                                 typename Acc<typename TnOp<MODE>::TL>::type* __restrict__ part) {
  typedef TnOp<MODE> O;
  typedef typename O::TA TA;
  typedef typename O::TL TL;
  typedef TileCfg<TL> C;
  typedef Mfma<TL> MF;
  typedef typename Acc<TL>::type TC;
  constexpr int NP = O::NP;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, LDK = BK + C::PAD;
  constexpr int VN = 16 / sizeof(TA);
  constexpr int AV = BK * BM / VN / 256, BV = BK * BN / VN / 256;
  constexpr int WTM = BM / 2, WTN = BN / 2, TI = WTM / 16, TJ = WTN / 16;
  __shared__ __align__(16) TL As[2][NP][BM * LDK];
  __shared__ __align__(16) TL Bs[2][NP][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int ti, tj, split;
  {
    int t;
    if (!tn_block(sym ? ntm * (ntm + 1) / 2 : ntm * ntn, kchunk, K, t, split)) return;
    if (sym) {
      ti = 0;
      int rowlen = ntm;
      while (t >= rowlen) { t -= rowlen; ti++; rowlen--; }
      tj = ti + t;
    } else {
      ti = t / ntn;
      tj = t % ntn;
    }
  }
  const int m0 = ti * BM, n0 = tj * BN;
  const int kbeg = split * kchunk, kend = min(K, kbeg + kchunk);
  const int Mv = (int)kp_roundup(M, VN), Nv = (int)kp_roundup(N, VN);
  TC* out = part + (long)split * M * N;

  TA va[AV][VN], vb[BV][VN];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AV; i++) {
      int v = tid + i * 256, kr = v / (BM / VN), mv = (v % (BM / VN)) * VN;
      int gk = k0 + kr, gm = m0 + mv;
      v16 x = {0u, 0u, 0u, 0u};
      if (gk < kend && gm < Mv) x = *(const v16*)(A + (long)gk * lda + gm);
      const TA* xe = (const TA*)&x;
      if (WEIGHTED) {
        const double wd = gk < kend ? rw[gk % rmod] : 0.0;
#pragma unroll
        for (int e = 0; e < VN; e++) va[i][e] = (TA)(to_d(xe[e]) * wd);
      } else {
#pragma unroll
        for (int e = 0; e < VN; e++) va[i][e] = xe[e];
      }
    }
#pragma unroll
    for (int i = 0; i < BV; i++) {
      int v = tid + i * 256, kr = v / (BN / VN), nv = (v % (BN / VN)) * VN;
      int gk = k0 + kr, gn = n0 + nv;
      v16 x = {0u, 0u, 0u, 0u};
      if (gk < kend && gn < Nv) x = *(const v16*)(B + (long)gk * ldb + gn);
      const TA* xe = (const TA*)&x;
#pragma unroll
      for (int e = 0; e < VN; e++) vb[i][e] = xe[e];
    }
  };
  auto put = [&](TL* plane0, TL* plane1, int idx, TA x) {
    if (NP == 2) {
      const TL hi = (TL)(float)x;
      plane0[idx] = hi;
      plane1[idx] = (TL)((float)x - (float)hi);
    } else {
      plane0[idx] = (TL)x;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AV; i++) {
      int v = tid + i * 256, kr = v / (BM / VN), mv = (v % (BM / VN)) * VN;
#pragma unroll
      for (int e = 0; e < VN; e++) put(As[buf][0], As[buf][NP - 1], (mv + e) * LDK + kr, va[i][e]);
    }
#pragma unroll
    for (int i = 0; i < BV; i++) {
      int v = tid + i * 256, kr = v / (BN / VN), nv = (v % (BN / VN)) * VN;
#pragma unroll
      for (int e = 0; e < VN; e++) put(Bs[buf][0], Bs[buf][NP - 1], (nv + e) * LDK + kr, vb[i][e]);
    }
  };

  typename MF::acc acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[i][j][e] = 0;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::K) {
      typename MF::frag a[NP][TI], b[NP][TJ];
#pragma unroll
      for (int h = 0; h < NP; h++) {
#pragma unroll
        for (int i = 0; i < TI; i++)
          a[h][i] = load_frag<TL>(&As[cur][h][(wm * WTM + i * 16) * LDK], lane, LDK, kk);
#pragma unroll
        for (int j = 0; j < TJ; j++)
          b[h][j] = load_frag<TL>(&Bs[cur][h][(wn * WTN + j * 16) * LDK], lane, LDK, kk);
      }
#pragma unroll
      for (int i = 0; i < TI; i++)
#pragma unroll
        for (int j = 0; j < TJ; j++) {
          acc[i][j] = MF::mma(a[0][i], b[0][j], acc[i][j]);
          if (NP == 2) {
            acc[i][j] = MF::mma(a[NP - 1][i], b[0][j], acc[i][j]);
            acc[i][j] = MF::mma(a[0][i], b[NP - 1][j], acc[i][j]);
          }
        }
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++) {
      const int col = n0 + wn * WTN + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int row = m0 + wm * WTM + i * 16 + MF::row(lane, e);
        if (row < M) out[(long)row * N + col] = (TC)acc[i][j][e];
      }
    }
}

// ---------------------------------------------------------------------------
// BF16x3 variant with the transpose done in registers.  A thread loads 8
// consecutive slab rows x 4 consecutive columns (eight 16-byte loads, 512 bytes
// contiguous per row across a half-wave), so for each of its 4 columns it holds
// 8 consecutive k; it splits them into BF16 hi and lo and writes each as one
// 16-byte LDS store into a k-contiguous [column][k] tile of 64-byte rows.
// A 16-byte access serves 16 lanes per LDS cycle over 256 bytes of banks, so
// both access patterns need 16 distinct (row mod 4, chunk) slots per group of
// 16 lanes: the fragment reads touch 16 consecutive columns at one chunk, the
// stores 16 columns 4 apart (one per column group) at one chunk.  Column c is
// kept in row c ^ ((c >> 2) & 3) and its chunk j at j ^ ((c >> 2) & 3) ^
// ((c >> 4) & 3), a bijection per row that separates both groups.
// Waves 0-1 load A, waves 2-3 load B.  Tile 128 x 128 x 32, four waves of
// 64 x 64, two LDS stages.
// ---------------------------------------------------------------------------
constexpr int X3_BM = 128, X3_BK = 32;

__device__ __forceinline__ int x3_pos(int col, int chunk) {
  const int q = (col >> 2) & 3;
  return (col ^ q) * X3_BK + ((chunk ^ q ^ ((col >> 4) & 3)) << 3);
}

// wsc[0] = 2^-e and wsc[1] = 2^e with max_i |rw[i]| < 2^e (1 and 1 when the weights
// are all zero or not finite): the scaling that keeps FP16 row weights within 1.
__device__ __forceinline__ void row_scale_at(const float* __restrict__ rw, int n,
                                             float* __restrict__ wsc) {
  __shared__ float part[4];
  float m = 0.0f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, fabsf(rw[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  m = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
  float s = 1.0f, u = 1.0f;
  if (m > 0.0f && m <= 3.0e38f) {
    int e;
    (void)frexpf(m, &e);   // m < 2^e
    s = ldexpf(1.0f, -e);
    u = ldexpf(1.0f, e);
  }
  wsc[0] = s;
  wsc[1] = u;
}
__global__ __launch_bounds__(256) void k_row_scale(const float* __restrict__ rw, int n,
                                                   float* __restrict__ wsc) {
  row_scale_at(rw, n, wsc);
}

// X3 = false: the single-pass FP16 variant (one FP16 plane, one MFMA per
// product) with the same tiles, loads and LDS layout.
template <bool WEIGHTED, bool X3>
__device__ __forceinline__ void tn_x3_at(const float* __restrict__ A, long lda,
                                         const float* __restrict__ B, long ldb, int M, int N,
                                         int K, const float* __restrict__ rw, int rmod, int sym,
                                         int ntm, int ntn, int kchunk, float* __restrict__ part,
                                         const float* __restrict__ wsc, int blk) {
  typedef typename std::conditional<X3, bf16, f16>::type TL;
  typedef typename std::conditional<X3, bf16x4, f16x4>::type TL4;
  typedef typename std::conditional<X3, bf16x8, f16x8>::type TL8;
  typedef Mfma<TL> MF;
  constexpr int BM = X3_BM, BK = X3_BK, TI = 4, TJ = 4, NPL = X3 ? 2 : 1;
  // [stage][operand][plane][BM * BK]
  __shared__ __align__(16) TL sm[2][2][NPL][BM * BK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int ti, tj, split;
  {
    int t;
    if (!tn_block(sym ? ntm * (ntm + 1) / 2 : ntm * ntn, kchunk, K, t, split, blk)) return;
    if (sym) {
      ti = 0;
      int rowlen = ntm;
      while (t >= rowlen) { t -= rowlen; ti++; rowlen--; }
      tj = ti + t;
    } else {
      ti = t / ntn;
      tj = t % ntn;
    }
  }
  const int m0 = ti * BM, n0 = tj * BM;
  const int kbeg = split * kchunk, kend = min(K, kbeg + kchunk);
  float* out = part + (long)split * M * N;
  // FP16: the row weights (residuals, any magnitude) enter scaled by the power of
  // two wsc[0] (k_row_scale: |w| <= 1) and the partial sums leave scaled by
  // wsc[1] = 1 / wsc[0]; both scalings are exact.  (The scaling is applied where
  // the weights are used, after the products: applied where they are loaded, it
  // would wait for those loads and with them for the prefetched rows.)
  float wscale = 1.0f, wunscale = 1.0f;
  if constexpr (WEIGHTED && !X3) {
    wscale = wsc[0];
    wunscale = wsc[1];
  }

  // loader role: operand (0 = A, 1 = B), column group, row group
  const int opd = tid >> 7, lt = tid & 127;
  const int cg = lt & 31, rg = lt >> 5;
  const float* src = opd == 0 ? A : B;
  const long ld = opd == 0 ? lda : ldb;
  const int col = (opd == 0 ? m0 : n0) + 4 * cg;
  const int lim = (int)kp_roundup(opd == 0 ? M : N, 4);
  const bool col_ok = col < lim;
  const int colc = col_ok ? col : 0;   // loads stay in bounds; masked lanes read column 0
  u32x4 ra[8];
  float wr[8];   // row weights of the A rows in flight (gradient)

#define KP_X3_LOAD(K0)                                                            \
  {                                                                              \
    _Pragma("unroll") for (int j = 0; j < 8; j++) {                              \
      const int gk = (K0) + 8 * rg + j;                                          \
      const int gkc = min(gk, kend - 1);                                         \
      ra[j] = ld16(src + (long)gkc * ld + colc);                                 \
      if (WEIGHTED && opd == 0) wr[j] = rw[gkc % rmod];                          \
    }                                                                            \
  }
#define KP_X3_STORE(BUF, K0)                                                      \
  {                                                                              \
    float wt[8];                                                                 \
    _Pragma("unroll") for (int j = 0; j < 8; j++) {                              \
      const int gk = (K0) + 8 * rg + j;                                          \
      wt[j] = (col_ok && gk < kend) ? 1.0f : 0.0f;                               \
      if (WEIGHTED && opd == 0) wt[j] *= wr[j] * wscale;                         \
    }                                                                            \
    f32x4 fr[8];                                                                 \
    _Pragma("unroll") for (int j = 0; j < 8; j++)                                \
      fr[j] = __builtin_bit_cast(f32x4, ra[j]) * wt[j];                          \
    _Pragma("unroll") for (int e = 0; e < 4; e++) {                              \
      f32x4 f0, f1;                                                              \
      _Pragma("unroll") for (int j = 0; j < 4; j++) {                            \
        f0[j] = fr[j][e];                                                        \
        f1[j] = fr[j + 4][e];                                                    \
      }                                                                          \
      const TL4 h0 = __builtin_convertvector(f0, TL4);                           \
      const TL4 h1 = __builtin_convertvector(f1, TL4);                           \
      const int pos = x3_pos(4 * cg + e, rg);                                    \
      TL8 hv = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);          \
      *(TL8*)&sm[BUF][opd][0][pos] = hv;                                         \
      if constexpr (X3) {                                                        \
        const TL4 l0 = __builtin_convertvector(f0 - __builtin_convertvector(h0, f32x4), TL4); \
        const TL4 l1 = __builtin_convertvector(f1 - __builtin_convertvector(h1, f32x4), TL4); \
        TL8 lv = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);        \
        *(TL8*)&sm[BUF][opd][NPL - 1][pos] = lv;                                 \
      }                                                                          \
    }                                                                            \
  }

  typename MF::acc acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[i][j][e] = 0;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    KP_X3_LOAD(kbeg);
    KP_X3_STORE(0, kbeg);
  }
  __syncthreads();
  const int fr = lane & 15, fc = lane >> 4;
  // uniform body: the last iteration also loads (clamped rows) and stores into
  // the unused stage, so the compiler sees no loads in flight at the loop head
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    const int knext = kbeg + (kt + 1) * BK;
    KP_X3_LOAD(knext);
    // keep the loads ahead of the products (the scheduler would sink them)
    __builtin_amdgcn_sched_barrier(0);
    typename MF::frag a[NPL][TI], b[NPL][TJ];
#pragma unroll
    for (int h = 0; h < NPL; h++) {
#pragma unroll
      for (int i = 0; i < TI; i++)
        a[h][i] = *(const TL8*)&sm[cur][0][h][x3_pos(wm * 64 + i * 16 + fr, fc)];
#pragma unroll
      for (int j = 0; j < TJ; j++)
        b[h][j] = *(const TL8*)&sm[cur][1][h][x3_pos(wn * 64 + j * 16 + fr, fc)];
    }
#pragma unroll
    for (int i = 0; i < TI; i++)
#pragma unroll
      for (int j = 0; j < TJ; j++) {
        acc[i][j] = MF::mma(a[0][i], b[0][j], acc[i][j]);
        if constexpr (X3) {
          acc[i][j] = MF::mma(a[NPL - 1][i], b[0][j], acc[i][j]);
          acc[i][j] = MF::mma(a[0][i], b[NPL - 1][j], acc[i][j]);
        }
      }
    __builtin_amdgcn_sched_barrier(0);
    KP_X3_STORE(cur ^ 1, knext);
    __syncthreads();
  }
#undef KP_X3_LOAD
#undef KP_X3_STORE

#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++) {
      const int c = n0 + wn * 64 + j * 16 + (lane & 15);
      if (c >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int r = m0 + wm * 64 + i * 16 + MF::row(lane, e);
        if (r < M) out[(long)r * N + c] = acc[i][j][e] * wunscale;
      }
    }
}
template <bool WEIGHTED, bool X3 = true>
__global__ __launch_bounds__(256) void k_tn_x3(const float* __restrict__ A, long lda,
                                               const float* __restrict__ B, long ldb, int M,
                                               int N, int K, const float* __restrict__ rw,
                                               int rmod, int sym, int ntm, int ntn, int kchunk,
                                               float* __restrict__ part,
                                               const float* __restrict__ wsc) {
  tn_x3_at<WEIGHTED, X3>(A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, wsc,
                         blockIdx.x);
}

template <int MODE>
static void launch_tn(dim3 g, const void* A, long lda, const void* B, long ldb, int M, int N, int K,
                      const double* rw, int rmod, bool sym, int ntm, int ntn, int kchunk,
                      void* part, hipStream_t st) {
  typedef typename TnOp<MODE>::TA TA;
  typedef typename Acc<typename TnOp<MODE>::TL>::type TC;
  if (rw)
    k_gemm_tn<MODE, true><<<g, 256, 0, st>>>((const TA*)A, lda, (const TA*)B, ldb, M, N, K, rw,
                                             rmod, sym, ntm, ntn, kchunk, (TC*)part);
  else
    k_gemm_tn<MODE, false><<<g, 256, 0, st>>>((const TA*)A, lda, (const TA*)B, ldb, M, N, K, rw,
                                              rmod, sym, ntm, ntn, kchunk, (TC*)part);
}

hipError_t gemm_tn_splitk(int mode, const void* A, long lda, const void* B, long ldb, int M, int N,
                          int K, const double* rw, const float* rwf, int rmod, bool sym,
                          void* part, int max_splits, int* splits_out, hipStream_t st,
                          float* wsc) {
  const int BT = (mode == M_F64) ? 64 : 128;
  const int BK = (mode == M_BF16 || mode == M_BF16X3 || mode == M_F16) ? 32 : 16;
  const int ntm = kp_cdiv(M, BT), ntn = kp_cdiv(N, BT);
  const int ntiles = sym ? ntm * (ntm + 1) / 2 : ntm * ntn;
  int splits = kp_cdiv(1024, ntiles);
  int max_by_k = kp_cdiv(K, 8 * BK);
  if (splits > max_by_k) splits = max_by_k;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  if (splits > 8) splits = std::min(max_splits, (int)kp_roundup(splits, 8));
  int kchunk = (int)kp_roundup(kp_cdiv(K, splits), BK);
  splits = kp_cdiv(K, kchunk);
  if (splits < 1) splits = 1;
  *splits_out = splits;
  // a linear grid in XCD-major order (see tn_block): 8 blocks per (tile, split group)
  dim3 g(8 * ntiles * kp_cdiv(splits, 8));
  switch (mode) {
    case M_F64: launch_tn<M_F64>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    case M_F32: launch_tn<M_F32>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    case M_BF16: launch_tn<M_BF16>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    case M_BF16X3:
      if (rw && !rwf) return hipErrorInvalidValue;
      if (rw)
        k_tn_x3<true><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, ldb, M, N, K, rwf,
                                         rmod, sym, ntm, ntn, kchunk, (float*)part, nullptr);
      else
        k_tn_x3<false><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, ldb, M, N, K,
                                          nullptr, rmod, sym, ntm, ntn, kchunk, (float*)part,
                                          nullptr);
      break;
    case M_F16:
      if (rw && (!rwf || !wsc)) return hipErrorInvalidValue;
      if (rw) {
        k_row_scale<<<1, 256, 0, st>>>(rwf, rmod, wsc);
        k_tn_x3<true, false><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, ldb, M, N,
                                                K, rwf, rmod, sym, ntm, ntn, kchunk,
                                                (float*)part, wsc);
      } else {
        k_tn_x3<false, false><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, ldb, M,
                                                 N, K, nullptr, rmod, sym, ntm, ntn, kchunk,
                                                 (float*)part, nullptr);
      }
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TP>
__device__ __forceinline__ void reduce_at(const TP* __restrict__ part, int splits, int M, int N,
                                          int sym, double* __restrict__ out, long so_m, long so_n,
                                          double alpha, double c_prev, long idx) {
  if (idx >= (long)M * N) return;
  int m = (int)(idx / N), n = (int)(idx % N);
  if (sym && n < m) return;
  double s = 0.0;
  for (int k = 0; k < splits; k++) s += (double)part[(long)k * M * N + idx];
  double* o = out + m * so_m + n * so_n;
  double v = alpha * s + (c_prev != 0.0 ? c_prev * *o : 0.0);
  *o = v;
  if (sym && n != m) {
    double* o2 = out + n * so_m + m * so_n;
    *o2 = v;   // the lower triangle equals the upper triangle before and after the update
  }
}
template <typename TP>
__global__ void k_reduce_splitk(const TP* __restrict__ part, int splits, int M, int N, int sym,
                                double* __restrict__ out, long so_m, long so_n, double alpha,
                                double c_prev) {
  reduce_at<TP>(part, splits, M, N, sym, out, so_m, so_n, alpha, c_prev,
                (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Grouped factor and gradient products (see GroupBlk): the split-K products of
// many instances in one launch, their reductions in another; the same bodies,
// split counts and tile orders as the single-instance launches.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T ld_uniform(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)p;
#else
  return *p;   // the host pass only parses device code
#endif
}

template <bool WEIGHTED, bool X3>
__global__ __launch_bounds__(256) void k_tn_x3_group(const TnJob* __restrict__ jobs,
                                                     const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const TnJob j = ld_uniform(jobs + g.job);
  tn_x3_at<WEIGHTED, X3>(j.A, j.lda, j.B, j.ldb, j.M, j.N, j.K, j.rw, j.rmod, j.sym, j.ntm, j.ntn,
                         j.kchunk, j.part, j.wsc, g.local);
}

__global__ __launch_bounds__(256) void k_reduce_group(const RedJob* __restrict__ jobs,
                                                      const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const RedJob j = ld_uniform(jobs + g.job);
  reduce_at<float>(j.part, j.splits, j.M, j.N, j.sym, j.out, j.so_m, j.so_n, j.alpha, j.c_prev,
                   (long)g.local * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_row_scale_group(const TnJob* __restrict__ jobs) {
  const TnJob j = ld_uniform(jobs + blockIdx.x);
  row_scale_at(j.rw, j.rmod, j.wsc);
}

bool make_tn_job(int mode, const float* A, long lda, const float* B, long ldb, int M, int N, int K,
                 const float* rwf, int rmod, bool sym, float* part, int max_splits, float* wsc,
                 TnJob* j, int* nblk) {
  if ((mode != M_BF16X3 && mode != M_F16) || M <= 0 || N <= 0 || K <= 0 ||
      (rwf && mode == M_F16 && !wsc))
    return false;
  // the split count and grid of gemm_tn_splitk
  const int BT = 128, BK = 32;
  const int ntm = kp_cdiv(M, BT), ntn = kp_cdiv(N, BT);
  const int ntiles = sym ? ntm * (ntm + 1) / 2 : ntm * ntn;
  int splits = kp_cdiv(1024, ntiles);
  int max_by_k = kp_cdiv(K, 8 * BK);
  if (splits > max_by_k) splits = max_by_k;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  if (splits > 8) splits = std::min(max_splits, (int)kp_roundup(splits, 8));
  const int kchunk = (int)kp_roundup(kp_cdiv(K, splits), BK);
  splits = kp_cdiv(K, kchunk);
  if (splits < 1) splits = 1;
  *j = TnJob{A, lda, B, ldb, M, N, K, rwf, rmod, sym ? 1 : 0, ntm, ntn, kchunk, part,
             mode == M_F16 ? wsc : nullptr, splits};
  *nblk = 8 * ntiles * kp_cdiv(splits, 8);
  return true;
}

RedJob make_red_job(const TnJob& t, double* out, long so_m, long so_n, double alpha,
                    double c_prev, int* nblk) {
  *nblk = kp_cdiv((long)t.M * t.N, 256);
  return RedJob{t.part, t.splits, t.M, t.N, t.sym, out, so_m, so_n, alpha, c_prev};
}

hipError_t tn_group(int mode, bool weighted, const TnJob* jobs, const GroupBlk* blk, int nblk,
                    hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  if (mode == M_BF16X3) {
    if (weighted) k_tn_x3_group<true, true><<<nblk, 256, 0, st>>>(jobs, blk);
    else k_tn_x3_group<false, true><<<nblk, 256, 0, st>>>(jobs, blk);
  } else if (mode == M_F16) {
    if (weighted) k_tn_x3_group<true, false><<<nblk, 256, 0, st>>>(jobs, blk);
    else k_tn_x3_group<false, false><<<nblk, 256, 0, st>>>(jobs, blk);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t row_scale_group(const TnJob* jobs, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  k_row_scale_group<<<njobs, 256, 0, st>>>(jobs);
  return hipGetLastError();
}

hipError_t reduce_group(const RedJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_reduce_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}

hipError_t reduce_splitk(int mode, const void* part, int splits, int M, int N, bool sym,
                         double* out, long so_m, long so_n, double alpha, double c_prev,
                         hipStream_t st) {
  long tot = (long)M * N;
  int nb = kp_cdiv(tot, 256);
  if (mode == M_F64)
    k_reduce_splitk<double><<<nb, 256, 0, st>>>((const double*)part, splits, M, N, sym, out,
                                                so_m, so_n, alpha, c_prev);
  else
    k_reduce_splitk<float><<<nb, 256, 0, st>>>((const float*)part, splits, M, N, sym, out, so_m,
                                               so_n, alpha, c_prev);
  return hipGetLastError();
}

}  // namespace kp
