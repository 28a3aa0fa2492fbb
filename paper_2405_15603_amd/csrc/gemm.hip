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

// XCD-aware tile order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs; remap so that each XCD receives a contiguous run of logical
// tiles (tiles that share slab rows then share one L2).
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int per = total / 8, rem = total % 8;
  const int x = b % 8, i = b / 8;
  // XCD x owns logical tiles [x*per + min(x, rem), ...) of length per + (x < rem)
  return x * per + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------------------
// part[s] = sum_{k in split s} w(k) A[k]^T B[k]   (A: K x M, B: K x N, rows)
// ---------------------------------------------------------------------------
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
  int ti, tj;
  {
    int t = blockIdx.x;
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
  const int split = blockIdx.y;
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
                          int K, const double* rw, int rmod, bool sym, void* part, int max_splits,
                          int* splits_out, hipStream_t st) {
  const int BT = (mode == M_F64) ? 64 : 128;
  const int BK = (mode == M_BF16 || mode == M_BF16X3) ? 32 : 16;
  const int ntm = kp_cdiv(M, BT), ntn = kp_cdiv(N, BT);
  const int ntiles = sym ? ntm * (ntm + 1) / 2 : ntm * ntn;
  int splits = kp_cdiv(1024, ntiles);
  int max_by_k = kp_cdiv(K, 8 * BK);
  if (splits > max_by_k) splits = max_by_k;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  int kchunk = (int)kp_roundup(kp_cdiv(K, splits), BK);
  splits = kp_cdiv(K, kchunk);
  if (splits < 1) splits = 1;
  *splits_out = splits;
  dim3 g(ntiles, splits);
  switch (mode) {
    case M_F64: launch_tn<M_F64>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    case M_F32: launch_tn<M_F32>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    case M_BF16: launch_tn<M_BF16>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    case M_BF16X3: launch_tn<M_BF16X3>(g, A, lda, B, ldb, M, N, K, rw, rmod, sym, ntm, ntn, kchunk, part, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TP>
__global__ void k_reduce_splitk(const TP* __restrict__ part, int splits, int M, int N, int sym,
                                double* __restrict__ out, long so_m, long so_n, double alpha,
                                double c_prev) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
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
