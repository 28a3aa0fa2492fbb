// Fused forward-Laplacian layer and its adjoint (Section 3.1, Eq.
// forward-laplacian-main; backward pass of Algorithm 1).
//
// Slabs are s-major: row s*N + p holds shared column s of point p (s = 0 value,
// 1..d first derivatives, S-1 the masked Laplacian).  For a fixed s the points
// are contiguous, so one layer is S products of an N x K block with the same
// weights.  A workgroup owns a tile of points x neurons and walks over s; the
// tanh quantities of each (point, neuron) -- t = tanh(a_value) and the running
// sum over derivative rows -- stay in the lane that holds that output, because
// every s produces the same MFMA output layout.  The s range is split in chunks
// (grid.y) for parallelism; a small finishing pass adds the chunk partials for
// the Laplacian row (forward) and the value row (backward), in a fixed order.
//
// Compute modes: FP64 and FP32 MFMA; BF16 MFMA (BF16 slabs and weights, used by
// the line search); BF16x3 (FP32 slabs split into BF16 hi + lo on the way into
// LDS, weights as BF16 hi + lo; acc += hi*hi + lo*hi + hi*lo), used by the
// mixed-precision curvature pass for FP32-level accuracy at BF16 MFMA rates.
#include <map>
#include <mutex>
#include <queue>
#include <tuple>

#include "common.h"
#include "fwdlap.h"
#include "launch.h"

namespace kp {

// ---------------------------------------------------------------------------
// MFMA policies
// ---------------------------------------------------------------------------
template <int MODE> struct Op;
template <> struct Op<M_F64> {
  typedef double TA;   // A in global memory
  typedef double TB;   // B in global memory
  typedef double TL;   // LDS element
  typedef double TC;   // compute / accumulate
  static constexpr int NA = 1, NB = 1, BK = 16, PAD = 2, VA = 2;
};
template <> struct Op<M_F32> {
  typedef float TA;
  typedef float TB;
  typedef float TL;
  typedef float TC;
  static constexpr int NA = 1, NB = 1, BK = 32, PAD = 4, VA = 4;
};
template <> struct Op<M_BF16> {
  typedef bf16 TA;
  typedef bf16 TB;
  typedef bf16 TL;
  typedef float TC;
  static constexpr int NA = 1, NB = 1, BK = 128, PAD = 8, VA = 8;
};
template <> struct Op<M_BF16X3> {
  typedef float TA;
  typedef bf16 TB;
  typedef bf16 TL;
  typedef float TC;
  static constexpr int NA = 2, NB = 2, BK = 64, PAD = 8, VA = 4;
};

// FP16: the slab operand is rounded once; the weights are split into FP16 hi + lo
// (two MFMAs per product), because their rounding error would be the same for
// every point and would not average out in the factor sums.  64-wide k-tiles: the
// register-staged loads keep one tile in flight, so a wider tile hides more of
// their latency (measured: the forward and adjoint products 12.1 -> 9.4 ms per step).
template <> struct Op<M_F16> {
  typedef float TA;
  typedef f16 TB;
  typedef f16 TL;
  typedef float TC;
  static constexpr int NA = 1, NB = 2, BK = 64, PAD = 8, VA = 4;
};

typedef uint4 v16;

template <typename TL>
__device__ __forceinline__ typename Mfma<TL>::frag frag_ld(const TL* base, int lane, int ldk, int k0);
template <>
__device__ __forceinline__ bf16x8 frag_ld<bf16>(const bf16* base, int lane, int ldk, int k0) {
  return *(const bf16x8*)(base + (lane & 15) * ldk + k0 + (lane >> 4) * 8);
}
template <>
__device__ __forceinline__ f16x8 frag_ld<f16>(const f16* base, int lane, int ldk, int k0) {
  return *(const f16x8*)(base + (lane & 15) * ldk + k0 + (lane >> 4) * 8);
}
template <>
__device__ __forceinline__ float frag_ld<float>(const float* base, int lane, int ldk, int k0) {
  return base[(lane & 15) * ldk + k0 + (lane >> 4)];
}
template <>
__device__ __forceinline__ double frag_ld<double>(const double* base, int lane, int ldk, int k0) {
  return base[(lane & 15) * ldk + k0 + (lane >> 4)];
}

__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int per = total / 8, rem = total % 8;
  const int x = b % 8, i = b / 8;
  return x * per + (x < rem ? x : rem) + i;
}

// Tile geometry: 8 waves as 4 (points) x 2 (neurons); wave tile WP x WN.  The
// backward kernel keeps three per-output values across s, so it uses the
// narrower wave tile (NARROW) to stay within registers.
constexpr int kThreads = 512;
template <int MODE, bool NARROW = false> struct Geo {
  static constexpr int NWP = 4, NWN = 2, NW = 8, NT = kThreads;
  static constexpr int WP = 32, WN = (MODE == M_F64 || NARROW) ? 32 : 64;
  static constexpr int BP = 4 * WP, BN = 2 * WN;
  static constexpr int TI = WP / 16, TJ = WN / 16;
};

template <int MODE, bool NARROW = false>
struct Mainloop {
  typedef Op<MODE> O;
  typedef Geo<MODE, NARROW> G;
  typedef typename O::TL TL;
  // FP16 forward products take 64-wide k-tiles (twice the products per round trip of
  // the register-staged loads); the narrow adjoint tile keeps 32 (more waves fit)
  static constexpr int BK = O::BK, LDK = BK + O::PAD;
  static constexpr int VA = O::VA;                  // A elements per 16-byte load
  static constexpr int VB = 16 / sizeof(typename O::TB);
  static constexpr int ANV = G::BP * (BK / VA), BNV = G::BN * (BK / VB);  // 16-byte vectors
  static constexpr int AV = (ANV + kThreads - 1) / kThreads;   // per thread (last may idle)
  static constexpr int BV = (BNV + kThreads - 1) / kThreads;
  struct Smem {
    TL a[2][O::NA][G::BP * LDK];
    TL b[2][O::NB][G::BN * LDK];
  };
};

// Software-pipelined walk over nsteps shared columns s (s = s_of(step)), each a
// product  A_s[p0:p0+BP, :K] * B[c0:c0+BN, :K]^T  accumulated in acc; the
// epilogue epi(step, s) runs when a column's product is complete.  The global
// loads of the next k-tile (also across columns) are in flight while the
// current one is multiplied; one barrier per k-tile.
// TRANS: the accumulators hold the transposed tile (MFMA rows are columns of B,
// MFMA columns are rows of A).
template <int MODE, bool NARROW, class SOf, class Epi, bool TRANS = false>
__device__ __forceinline__ void sloop(typename Mainloop<MODE, NARROW>::Smem& sm,
                                      const typename Op<MODE>::TA* __restrict__ A, long lda,
                                      int N, int p0, const typename Op<MODE>::TB* __restrict__ B,
                                      const typename Op<MODE>::TB* __restrict__ B2, long ldb,
                                      int c0, int ncols, int K, int nsteps, SOf s_of, Epi epi) {
  typedef Mainloop<MODE, NARROW> ML;
  typedef Op<MODE> O;
  typedef Geo<MODE, NARROW> G;
  typedef typename O::TL TL;
  typedef Mfma<TL> MF;
  constexpr int BK = ML::BK, LDK = ML::LDK, VA = ML::VA, VB = ML::VB;
  constexpr int AV = ML::AV, BV = ML::BV, NB = O::NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wp = wave >> 1, wn = wave & 1;
  // per-thread load coordinates (fixed for the whole loop)
  int ar[AV], ak[AV], br[BV], bk[BV];
#pragma unroll
  for (int i = 0; i < AV; i++) {
    const int v = tid + i * kThreads;
    ar[i] = v < ML::ANV ? v / (BK / VA) : 1 << 20;
    ak[i] = (v % (BK / VA)) * VA;
  }
#pragma unroll
  for (int i = 0; i < BV; i++) {
    const int v = tid + i * kThreads;
    br[i] = v < ML::BNV ? v / (BK / VB) : 1 << 20;   // out-of-tile: never loaded or stored
    bk[i] = (v % (BK / VB)) * VB;
  }
  u32x4 ra[AV], rb[NB][BV];
  const u32x4 z16 = {0u, 0u, 0u, 0u};

#define KP_GLOAD(AROW0, K0)                                                           \
  {                                                                                   \
    _Pragma("unroll") for (int i = 0; i < AV; i++) {                                  \
      const int p = p0 + ar[i], k = (K0) + ak[i];                                     \
      ra[i] = (p < N && k < K) ? ld16(A + ((AROW0) + p) * lda + k) : z16;             \
    }                                                                                 \
    _Pragma("unroll") for (int i = 0; i < BV; i++) {                                  \
      const int c = c0 + br[i], k = (K0) + bk[i];                                     \
      const bool ok = c < ncols && k < K;                                             \
      rb[0][i] = ok ? ld16(B + (long)c * ldb + k) : z16;                              \
      if constexpr (NB == 2) rb[NB - 1][i] = ok ? ld16(B2 + (long)c * ldb + k) : z16; \
    }                                                                                 \
  }
#define KP_SSTORE(BUF)                                                                \
  {                                                                                   \
    _Pragma("unroll") for (int i = 0; i < AV; i++) {                                  \
      if (ar[i] >= G::BP) continue;                                                   \
      if constexpr (MODE == M_BF16X3) {                                               \
        const f32x4 fv = __builtin_bit_cast(f32x4, ra[i]);                            \
        const bf16x4 hv = __builtin_convertvector(fv, bf16x4);                        \
        const bf16x4 lv =                                                             \
            __builtin_convertvector(fv - __builtin_convertvector(hv, f32x4), bf16x4); \
        *(bf16x4*)(&sm.a[BUF][0][ar[i] * LDK + ak[i]]) = hv;                          \
        *(bf16x4*)(&sm.a[BUF][O::NA - 1][ar[i] * LDK + ak[i]]) = lv;                  \
      } else if constexpr (MODE == M_F16) {                                           \
        const f32x4 fv = __builtin_bit_cast(f32x4, ra[i]);                            \
        *(f16x4*)(&sm.a[BUF][0][ar[i] * LDK + ak[i]]) = __builtin_convertvector(fv, f16x4); \
      } else {                                                                        \
        *(u32x4*)(&sm.a[BUF][0][ar[i] * LDK + ak[i]]) = ra[i];                        \
      }                                                                               \
    }                                                                                 \
    _Pragma("unroll") for (int i = 0; i < BV; i++) {                                  \
      if (br[i] >= G::BN) continue;                                                   \
      _Pragma("unroll") for (int h = 0; h < NB; h++)                                  \
        *(u32x4*)(&sm.b[BUF][h][br[i] * LDK + bk[i]]) = rb[h][i];                     \
    }                                                                                 \
  }

  typename MF::acc acc[G::TI][G::TJ];
#pragma unroll
  for (int i = 0; i < G::TI; i++)
#pragma unroll
    for (int j = 0; j < G::TJ; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[i][j][e] = 0;
  const int nk = (K + BK - 1) / BK;
  const int total = nsteps * nk;
  if (total <= 0) return;
  KP_GLOAD((long)s_of(0) * N, 0);
  KP_SSTORE(0);
  __syncthreads();
  int st = 0, kt = 0;
  for (int g = 0; g < total; g++) {
    const int cur = g & 1;
    const bool more = g + 1 < total;
    if (more) {
      const int nkt = kt + 1 == nk ? 0 : kt + 1;
      const int nst = kt + 1 == nk ? st + 1 : st;
      KP_GLOAD((long)s_of(nst) * N, nkt * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::K) {
      typename MF::frag a[O::NA][G::TI], b[NB][G::TJ];
#pragma unroll
      for (int h = 0; h < O::NA; h++)
#pragma unroll
        for (int i = 0; i < G::TI; i++)
          a[h][i] = frag_ld<TL>(&sm.a[cur][h][(wp * G::WP + i * 16) * LDK], lane, LDK, kk);
#pragma unroll
      for (int h = 0; h < NB; h++)
#pragma unroll
        for (int j = 0; j < G::TJ; j++)
          b[h][j] = frag_ld<TL>(&sm.b[cur][h][(wn * G::WN + j * 16) * LDK], lane, LDK, kk);
#pragma unroll
      for (int i = 0; i < G::TI; i++)
#pragma unroll
        for (int j = 0; j < G::TJ; j++) {
          if constexpr (TRANS) {
            acc[i][j] = MF::mma(b[0][j], a[0][i], acc[i][j]);
            if constexpr (MODE == M_BF16X3) {
              acc[i][j] = MF::mma(b[0][j], a[O::NA - 1][i], acc[i][j]);
              acc[i][j] = MF::mma(b[NB - 1][j], a[0][i], acc[i][j]);
            } else if constexpr (MODE == M_F16) {
              acc[i][j] = MF::mma(b[NB - 1][j], a[0][i], acc[i][j]);
            }
          } else {
            acc[i][j] = MF::mma(a[0][i], b[0][j], acc[i][j]);
            if constexpr (MODE == M_BF16X3) {
              acc[i][j] = MF::mma(a[O::NA - 1][i], b[0][j], acc[i][j]);
              acc[i][j] = MF::mma(a[0][i], b[NB - 1][j], acc[i][j]);
            } else if constexpr (MODE == M_F16) {
              acc[i][j] = MF::mma(a[0][i], b[NB - 1][j], acc[i][j]);
            }
          }
        }
    }
    if (kt + 1 == nk) {
      epi(st, s_of(st), acc);
#pragma unroll
      for (int i = 0; i < G::TI; i++)
#pragma unroll
        for (int j = 0; j < G::TJ; j++)
#pragma unroll
          for (int e = 0; e < 4; e++) acc[i][j][e] = 0;
      kt = 0;
      st++;
    } else {
      kt++;
    }
    if (more) KP_SSTORE(cur ^ 1);
    __syncthreads();
  }
#undef KP_GLOAD
#undef KP_SSTORE
}

// ---------------------------------------------------------------------------
// Direct-to-LDS variant of sloop for operands used as stored (BF16, FP32, FP64):
// every k-tile row is 128 bytes (8 chunks of 16 B), loaded with
// global_load_lds_dwordx4 into a ring of kStages stages, kStages-1 tiles in
// flight.  A pass covers NS shared columns s at once: a stage holds NS A tiles
// and one B tile, so the weights are fetched once per NS products.  A wave's
// load instruction fills 1 KB = 8 rows; chunk q of row r sits at chunk position
// q ^ ((r >> 1) & 7), which makes the 16-row fragment reads conflict-free.
// Chunks outside the valid rows / k range are redirected to a valid address:
// rows past N or ncols only feed discarded outputs, and chunks past K read a
// 16-byte zero block.  K must be a multiple of 16 bytes.  The accumulators hold
// the transposed tile: acc[q][i][j] = B_j A_{q,i}^T, i.e. MFMA rows are neurons
// and MFMA columns are points.  epi(step, s, acc[q]) runs for the steps of a
// pass in order once its products are complete.
// ---------------------------------------------------------------------------
__device__ __align__(16) u32x4 kZeroChunk = {0u, 0u, 0u, 0u};

// Geometry of the direct-to-LDS forward kernel: NWP x NWN waves, each owning a
// WP (points) x WN (neurons) tile; NS shared columns per pass; ST ring stages.
// A wide neuron tile (256) reads each point tile's slab rows fewer times, and
// four columns per pass amortise the epilogue and its store drain; with two
// stages the ring is 128 KB.  Measured against 128 x 128 tiles, two or three
// columns per pass, three or four stages and 64-byte k-tiles, this is the
// fastest.
template <int NWP_, int NWN_, int NS_> struct DGeoT {
  static constexpr int NWP = NWP_, NWN = NWN_, WP = 32, WN = 64, NS = NS_, ST = 2;
  static constexpr int RB = 128;   // bytes of a k-tile row (64-byte rows with more stages were slower)
  static constexpr int NW = NWP * NWN, NT = 64 * NW;
  static constexpr int BP = NWP * WP, BN = NWN * WN;
  static constexpr int TI = WP / 16, TJ = WN / 16;
};
template <int MODE> struct DGeo;
template <> struct DGeo<M_BF16> : DGeoT<2, 4, 4> {};
// Narrower neuron tiles for narrow layers (the grouped line search of many small
// networks): the same wave tile, waves stacked along the points.  128 x 128 with
// four rows per pass fills the 160 KB of LDS with its two-stage ring; 256 x 64
// holds two rows per pass.  An output element's products and sums are the same
// in every geometry.
using DGeoW128 = DGeoT<4, 2, 4>;
using DGeoW64 = DGeoT<8, 1, 2>;

template <class G, typename T>
struct DmaCfg {
  static constexpr int RB = G::RB;                    // row bytes: 128 or 64
  static constexpr int CPR = RB / 16;                 // 16-byte chunks per row
  static constexpr int RPI = 1024 / RB;               // rows per 1 KB load instruction
  static constexpr int E = 16 / sizeof(T);            // elements per chunk
  static constexpr int BK = RB / sizeof(T);           // k per tile
  static constexpr int ACH = G::BP / RPI, BCH = G::BN / RPI;   // 1 KB chunks per tile
  static constexpr int NCH = G::NS * ACH + BCH;
  static constexpr int PER_WAVE = NCH / G::NW;
  static constexpr int STAGE = NCH * 1024;             // bytes
  static_assert(ACH % G::NW == 0 && BCH % G::NW == 0,
                "every wave issues the same number of chunk loads of one operand");
};
template <int MODE> constexpr bool kDma = MODE == M_BF16;

// Chunk position of chunk q in row r: q ^ swz(r).  Rows of 128 B (8 chunks)
// repeat the bank pattern every 2 rows, rows of 64 B (4 chunks) every 4 rows; the
// XOR spreads a 16-row fragment over distinct banks.
template <int RB> __device__ __forceinline__ int swz(int r) {
  return RB == 128 ? ((r >> 1) & 7) : ((r >> 2) & 3);
}

template <typename TL, int RB>
__device__ __forceinline__ typename Mfma<TL>::frag frag_dma(const char* tile, int lane, int kk);
// bf16: 8 consecutive k of row lane%16 starting at kk + 8*(lane/16)
template <>
__device__ __forceinline__ bf16x8 frag_dma<bf16, 128>(const char* tile, int lane, int kk) {
  const int r = lane & 15, c = (kk >> 3) + (lane >> 4);
  return *(const bf16x8*)(tile + r * 128 + ((c ^ swz<128>(r)) << 4));
}
template <>
__device__ __forceinline__ bf16x8 frag_dma<bf16, 64>(const char* tile, int lane, int kk) {
  const int r = lane & 15, c = (kk >> 3) + (lane >> 4);
  return *(const bf16x8*)(tile + r * 64 + ((c ^ swz<64>(r)) << 4));
}

template <int MODE, class G, class SOf, class Epi>
__device__ __forceinline__ void sloop_dma(char* lds, const typename Op<MODE>::TL* __restrict__ A,
                                          long lda, int N, int p0,
                                          const typename Op<MODE>::TL* __restrict__ B, long ldb,
                                          int c0, int ncols, int K, int nsteps, SOf s_of,
                                          Epi epi) {
  typedef typename Op<MODE>::TL TL;
  typedef DmaCfg<G, TL> D;
  typedef Mfma<TL> MF;
  constexpr int NS = G::NS, kStages = G::ST, NW = G::NW;
  constexpr int E = D::E, BK = D::BK;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wp = wave / G::NWN, wn = wave % G::NWN;
  const int nk = (K + BK - 1) / BK;
  const int npass = (nsteps + NS - 1) / NS;
  const int total = npass * nk;
  if (total <= 0) return;
  constexpr int RB = D::RB;
  const int rin = lane / D::CPR, pos = lane % D::CPR;

  // Per-thread chunk coordinates are fixed for the whole loop: chunk slot j
  // (q = wave + NW j) belongs to A tile j / (ACH / NW) or, past NS A tiles, to B.
  constexpr int JA = NS * D::ACH / NW;   // slots 0..JA-1 load A tiles, the rest B
  int off[D::PER_WAVE], kin[D::PER_WAVE];   // element offset (without k0), chunk k offset
#pragma unroll
  for (int j = 0; j < D::PER_WAVE; j++) {
    const int q = wave + NW * j;
    if (j < JA) {
      const int r = (q % D::ACH) * D::RPI + rin;
      kin[j] = (pos ^ swz<RB>(r)) * E;
      off[j] = min(p0 + r, N - 1) * (int)lda + kin[j];
    } else {
      const int r = (q - NS * D::ACH) * D::RPI + rin;
      kin[j] = (pos ^ swz<RB>(r)) * E;
      off[j] = min(c0 + r, ncols - 1) * (int)ldb + kin[j];
    }
  }
  const TL* zchunk = (const TL*)&kZeroChunk;

  // Issue the loads of the next tile in order (tile index gi = pass ips, k-tile
  // ikt, stage ist); counters advance instead of dividing by nk.
  int ips = 0, ikt = 0, ist = 0;
  long sbase[NS];
  int i_k0 = 0;
  bool i_last = false;   // only the last k-tile has chunks past K
  char* i_stage = lds;
  auto issue_begin = [&]() {
    if (ikt == 0) {
#pragma unroll
      for (int q = 0; q < NS; q++) sbase[q] = (long)s_of(min(ips * NS + q, nsteps - 1)) * N * lda;
    }
    i_k0 = ikt * BK;
    i_last = i_k0 + BK > K;
    i_stage = lds + ist * D::STAGE;
  };
  auto issue_slot = [&](int j) {
    const TL* src = j < JA ? A + sbase[j / (D::ACH / NW)] + off[j] + i_k0 : B + off[j] + i_k0;
    if (i_last) src = i_k0 + kin[j] < K ? src : zchunk;
    __builtin_amdgcn_global_load_lds((const KP_GLOBAL void*)src,
                                     (__attribute__((address_space(3))) void*)(i_stage +
                                                                               (wave + NW * j) * 1024),
                                     16, 0, 0);
  };
  auto issue_end = [&]() {
    if (++ikt == nk) { ikt = 0; ips++; }
    if (++ist == kStages) ist = 0;
  };
  auto issue = [&]() {
    issue_begin();
#pragma unroll
    for (int j = 0; j < D::PER_WAVE; j++) issue_slot(j);
    issue_end();
  };

  typename MF::acc acc[NS][G::TI][G::TJ];
#pragma unroll
  for (int q = 0; q < NS; q++)
#pragma unroll
    for (int i = 0; i < G::TI; i++)
#pragma unroll
      for (int j = 0; j < G::TJ; j++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[q][i][j][e] = 0;

  for (int g = 0; g < kStages - 1 && g < total; g++) issue();
  int ps = 0, kt = 0, cst = 0;
  bool drained = false;   // stores were issued: wait for everything
  for (int g = 0; g < total; g++) {
    // tile g must have landed: at most (tiles after g in flight) * PER_WAVE loads pending
    const int after = min(kStages - 2, total - 1 - g);
    static_assert(kStages >= 2 && kStages <= 4, "up to two tiles in flight behind this one");
    if (drained || after <= 0) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    } else if (after == 1) {
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(D::PER_WAVE) : "memory");
    } else {
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"(D::PER_WAVE * (kStages > 3 ? 2 : 1)) : "memory");
    }
    drained = false;
    // The waits above cover this wave's loads and the barrier the other waves'
    // (and their reads of the stage refilled next).  A plain s_barrier: a
    // workgroup fence would drain every load in flight.  The memory clobber
    // keeps the compiler from moving LDS accesses across it.
    asm volatile("s_barrier" ::: "memory");
    // The next tile's loads are spread over the product groups below (one slot
    // after each group) rather than issued together, so that no wave waits at
    // the barrier's exit for the address unit to accept a burst of loads
    // (measured: issuing them all in the first half of the groups is slower).
    const bool nxt = g + kStages - 1 < total;
    if (nxt) issue_begin();
    const char* stage = lds + cst * D::STAGE;
    if (++cst == kStages) cst = 0;
    const char* Bt = stage + NS * D::ACH * 1024 + (wn * G::WN) * RB;
    const bool two = NS == 1 || ps * NS + 1 < nsteps;   // second column of the pass is real
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::K) {
      typename MF::frag b[G::TJ];
#pragma unroll
      for (int j = 0; j < G::TJ; j++) b[j] = frag_dma<TL, RB>(Bt + j * 16 * RB, lane, kk);
#pragma unroll
      for (int q = 0; q < NS; q++) {
        if (q == 0 || two) {
          const char* At = stage + q * D::ACH * 1024 + (wp * G::WP) * RB;
          typename MF::frag a[G::TI];
#pragma unroll
          for (int i = 0; i < G::TI; i++) a[i] = frag_dma<TL, RB>(At + i * 16 * RB, lane, kk);
#pragma unroll
          for (int i = 0; i < G::TI; i++)
#pragma unroll
            for (int j = 0; j < G::TJ; j++) acc[q][i][j] = MF::mma(b[j], a[i], acc[q][i][j]);
        }
        if (nxt) {
          constexpr int NG = (BK / MF::K) * NS;
          const int grp = (kk / MF::K) * NS + q;
#pragma unroll
          for (int j = grp; j < D::PER_WAVE; j += NG) issue_slot(j);
        }
      }
    }
    if (nxt) issue_end();
    if (kt + 1 == nk) {
#pragma unroll
      for (int q = 0; q < NS; q++) {
        const int st = ps * NS + q;
        if (st < nsteps) epi(st, s_of(st), acc[q]);
#pragma unroll
        for (int i = 0; i < G::TI; i++)
#pragma unroll
          for (int j = 0; j < G::TJ; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[q][i][j][e] = 0;
      }
      drained = true;
      kt = 0;
      ps++;
    } else {
      kt++;
    }
  }
  __syncthreads();
}

// Weight of derivative row i in the second-order row (1 or 0 for a Laplacian
// over a subset of the coordinates), read through the scalar cache (the weights
// are read-only during a launch).
__device__ __forceinline__ float wt_at(const float* wts, int i) {
  return ((const __attribute__((address_space(4))) float*)wts)[i];
}
// The weight in the compute type: FP64 work reads the FP64 copy (eigenvalues of
// a coefficient matrix are not exact in FP32).
template <typename TC, typename Args>
__device__ __forceinline__ TC wt_of(const Args& a, int i) {
  if constexpr (std::is_same<TC, double>::value)
    return ((const __attribute__((address_space(4))) double*)a.wts64)[i];
  else
    return (TC)wt_at(a.wts, i);
}

// ---------------------------------------------------------------------------
// Forward layer.  Chunk c of C handles derivative rows [1 + c*len, ...), always
// recomputes the value row (s = 0) first for t, and the last chunk also forms the
// Laplacian row's pre-activation.  Outputs: z rows (value, derivatives) of the
// next slab, optional pre-activations, and the tables for the finishing pass.
// ---------------------------------------------------------------------------
template <int MODE>
using FwdGeo = typename std::conditional<kDma<MODE>, DGeo<M_BF16>, Geo<MODE>>::type;

template <class G> constexpr int dma_smem() { return G::ST * DmaCfg<G, bf16>::STAGE; }
static_assert(dma_smem<DGeoW128>() <= 160 * 1024 && dma_smem<DGeoW64>() <= 160 * 1024,
              "the ring fits the LDS of a compute unit");
template <int MODE> constexpr int fwd_smem() {
  if constexpr (kDma<MODE>)
    return dma_smem<DGeo<M_BF16>>();
  else
    return (int)sizeof(typename Mainloop<MODE>::Smem);
}

// One workgroup of a layer product: tile t, chunk `chunk` of nch.  PLAIN: rows
// without derivative or Laplacian rows (one column per point, no tables).
template <int MODE, typename TZ, bool A4, bool PLAIN = false, class G = FwdGeo<MODE>>
__device__ __forceinline__ void fwd_block(const FwdLayerArgs& a, int t, int chunk, int nch,
                                          char* smem) {
  typedef Op<MODE> O;
  typedef typename O::TC TC;
  typedef typename O::TL TL;
  typedef Mfma<TL> MF;
  // The direct-to-LDS loop computes the transposed tile (neurons x points), so a
  // lane holds four consecutive neurons of one point and, when every output row
  // is 4-aligned (A4), stores them as one vector.
  constexpr bool TR = kDma<MODE> || MODE != M_F64;   // FP64 MFMA rows are not consecutive
  constexpr bool VEC = TR && A4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wp = wave / G::NWN, wn = wave % G::NWN;
  const int ntc = (a.h_out + G::BN - 1) / G::BN;
  const int ntp = (a.N + G::BP - 1) / G::BP;
  const int p0 = (t / ntc) * G::BP, c0 = (t % ntc) * G::BN;
  const int nd = a.nd;
  const int len = (nd + nch - 1) / nch;
  const int dbeg = 1 + chunk * len, dend = min(1 + nd, dbeg + len);
  const int nder = (PLAIN || a.value_only) ? 0 : max(0, dend - dbeg);
  const bool lap_here = !PLAIN && a.has_lap && !a.value_only && chunk == nch - 1;
  const int nsteps = 1 + nder + (lap_here ? 1 : 0);
  const int S = a.S;
  // output coordinates of accumulator element (i, j, e)
  auto P = [&](int i, int e) {
    return p0 + wp * G::WP + i * 16 + (TR ? (lane & 15) : MF::row(lane, e));
  };
  auto Cn = [&](int j, int e) {
    return c0 + wn * G::WN + j * 16 + (TR ? MF::row(lane, e) : (lane & 15));
  };

  TC tv[G::TI][G::TJ][4], sq[G::TI][G::TJ][4];
#pragma unroll
  for (int i = 0; i < G::TI; i++)
#pragma unroll
    for (int j = 0; j < G::TJ; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) { sq[i][j][e] = 0; tv[i][j][e] = 0; }

  // step 0: value row, steps 1..nder: derivative rows of this chunk, then the Laplacian row
  auto s_of = [=](int st) { return st == 0 ? 0 : (st <= nder ? dbeg + st - 1 : S - 1); };
  // Vector path: per-lane row and per-group neuron predicates; the column kind is
  // uniform, so each kind has its own loop over the tile.  With BF16 rows, s1 =
  // 1 - t^2 of the value row is kept in half precision (relative rounding 2^-11,
  // below the 2^-9 of the BF16 rows it scales), which leaves the main loop the
  // registers it needs; FP32 rows keep it in FP32.
  constexpr bool kBf = std::is_same<TZ, bf16>::value;
  typedef typename std::conditional<kBf, f16x4, f32x4>::type S1V;
  auto store4z = [](TZ* dst, const f32x4& v) {
    if constexpr (kBf)
      *gmem((bf16x4*)dst) = __builtin_convertvector(v, bf16x4);
    else
      *gmem((f32x4*)dst) = v;
  };
  S1V s1h[G::TI][G::TJ];
  bool p_ok[G::TI], c_ok[G::TJ];
#pragma unroll
  for (int i = 0; i < G::TI; i++) p_ok[i] = P(i, 0) < a.N;
#pragma unroll
  for (int j = 0; j < G::TJ; j++) c_ok[j] = Cn(j, 0) < a.h_out;
  auto epi_vec = [&](int s, typename MF::acc (&acc)[G::TI][G::TJ]) {
    if constexpr (VEC) {
      const bool is_d = s >= 1 && s <= nd;
      const int kind = s == 0 ? 0 : (is_d ? 1 : 2);
      const bool keep = !a.sparse_store || (kind == 0 ? a.keep_value != 0
                                                      : (s >= a.keep_lo && s <= a.keep_hi));
      const long rbase = (long)s * a.N + P(0, 0);
      const int cb0 = Cn(0, 0);
      auto zrow = [&](int i) { return (TZ*)a.z + (rbase + i * 16) * a.ldzo + cb0; };
      auto prow = [&](int i) { return (TC*)a.pre + (rbase + i * 16) * a.ldp + cb0; };
      auto tabrow = [&](void* tab, int i) {
        return (TC*)tab + (long)(P(0, 0) + i * 16) * a.h_out + cb0;
      };
      if (kind == 1) {
        const float wk = wt_at(a.wts, s - 1);
        if (wk != 0.0f) {
#pragma unroll
          for (int i = 0; i < G::TI; i++)
#pragma unroll
            for (int j = 0; j < G::TJ; j++)
#pragma unroll
              for (int e = 0; e < 4; e++) sq[i][j][e] += (wk * acc[i][j][e]) * acc[i][j][e];
        }
        if (keep) {
#pragma unroll
          for (int i = 0; i < G::TI; i++)
#pragma unroll
            for (int j = 0; j < G::TJ; j++) {
              const f32x4 o = __builtin_convertvector(s1h[i][j], f32x4) * (f32x4)acc[i][j];
              if (p_ok[i] && c_ok[j])
                store4z(zrow(i) + j * 16, o);
            }
        }
        if (a.pre) {
#pragma unroll
          for (int i = 0; i < G::TI; i++)
#pragma unroll
            for (int j = 0; j < G::TJ; j++)
              if (p_ok[i] && c_ok[j]) *gmem((f32x4*)(prow(i) + j * 16)) = acc[i][j];
        }
      } else if (kind == 0) {
        const bool first = chunk == 0;
#pragma unroll
        for (int i = 0; i < G::TI; i++)
#pragma unroll
          for (int j = 0; j < G::TJ; j++) {
            f32x4 t, s1;
#pragma unroll
            for (int e = 0; e < 4; e++) {
              t[e] = act_tanh(acc[i][j][e]);
              s1[e] = __builtin_fmaf(-t[e], t[e], 1.0f);
            }
            s1h[i][j] = __builtin_convertvector(s1, S1V);
            if (first && p_ok[i] && c_ok[j]) {
              if (keep) store4z(zrow(i) + j * 16, t);
              if (a.pre) *gmem((f32x4*)(prow(i) + j * 16)) = acc[i][j];
              if (a.tab_t) *gmem((f32x4*)(tabrow(a.tab_t, i) + j * 16)) = t;
            }
          }
      } else {
#pragma unroll
        for (int i = 0; i < G::TI; i++)
#pragma unroll
          for (int j = 0; j < G::TJ; j++)
            if (p_ok[i] && c_ok[j]) {
              if (a.pre) *gmem((f32x4*)(prow(i) + j * 16)) = acc[i][j];
              *gmem((f32x4*)(tabrow(a.tab_lap, i) + j * 16)) = acc[i][j];
            }
      }
    }
  };
  auto epi = [&](int st, int s, typename MF::acc (&acc)[G::TI][G::TJ]) {
    if constexpr (VEC) {
      epi_vec(s, acc);
      return;
    }
    const bool is_d = s >= 1 && s <= nd;
    const TC m = is_d ? wt_of<TC>(a, s - 1) : (TC)0;
    const int kind = s == 0 ? 0 : (is_d ? 1 : 2);
    // whether this z row is stored (the Laplacian row is finished separately)
    const bool keep = !a.sparse_store || (kind == 0 ? a.keep_value != 0
                                                    : (s >= a.keep_lo && s <= a.keep_hi));
#pragma unroll
    for (int i = 0; i < G::TI; i++)
#pragma unroll
      for (int j = 0; j < G::TJ; j++) {
        TC v[4], out[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          v[e] = (TC)acc[i][j][e];
          if (kind == 0) {
            out[e] = act_tanh(v[e]);
            tv[i][j][e] = out[e];
          } else if (kind == 1) {
            const TC th = tv[i][j][e];
            sq[i][j][e] += m * v[e] * v[e];
            out[e] = ((TC)1 - th * th) * v[e];
          }
        }
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int p = P(i, e), c = Cn(j, e);
          if (p >= a.N || c >= a.h_out) continue;
          const long row = (long)s * a.N + p;
          if (kind == 0 && chunk != 0) continue;
          if (kind <= 1 && keep) ((TZ*)a.z)[row * a.ldzo + c] = cvt<TZ>((double)out[e]);
          if (a.pre) ((TC*)a.pre)[row * a.ldp + c] = v[e];
          if (kind == 0 && a.tab_t) ((TC*)a.tab_t)[(long)p * a.h_out + c] = out[e];
          if (kind == 2) ((TC*)a.tab_lap)[(long)p * a.h_out + c] = v[e];
        }
      }
  };
  if constexpr (kDma<MODE>)
    sloop_dma<MODE, G>(smem, (const TL*)a.zin, a.ldz, a.N, p0, (const TL*)a.w, a.ldw, c0,
                       a.h_out, a.kz > 0 ? a.kz : a.K, nsteps, s_of, epi);
  else
    sloop<MODE, false, decltype(s_of), decltype(epi), TR>(
        *(typename Mainloop<MODE>::Smem*)smem, (const typename O::TA*)a.zin, a.ldz, a.N, p0,
        (const typename O::TB*)a.w, (const typename O::TB*)a.w2, a.ldw, c0, a.h_out, a.K, nsteps,
        s_of, epi);
  if (a.has_lap) {
#pragma unroll
    for (int i = 0; i < G::TI; i++)
#pragma unroll
      for (int j = 0; j < G::TJ; j++) {
        if constexpr (VEC) {
          if (p_ok[i] && c_ok[j])
            *gmem((f32x4*)((TC*)a.tab_sq + ((long)chunk * a.N + P(i, 0)) * a.h_out + Cn(j, 0))) =
                f32x4{(float)sq[i][j][0], (float)sq[i][j][1], (float)sq[i][j][2], (float)sq[i][j][3]};
        } else {
#pragma unroll
          for (int e = 0; e < 4; e++) {
            const int p = P(i, e), c = Cn(j, e);
            if (p < a.N && c < a.h_out)
              ((TC*)a.tab_sq)[((long)chunk * a.N + p) * a.h_out + c] = sq[i][j][e];
          }
        }
      }
  }
}

// Grid (tiles0 + tiles1) x nch: blocks x < tiles0 take the tiles of layer
// product a0 in chunk y; blocks x >= tiles0 of chunk 0 take the tiles of a1, a
// second point set of the same layer without derivative rows (the boundary
// points), in one chunk; the other blocks return at once.  The two sets take
// separate inlined copies of the block, so neither pays registers for choosing
// between them.
template <int MODE, typename TZ, bool A4 = false>
__global__ __launch_bounds__(FwdGeo<MODE>::NT) void k_fwdlap(FwdLayerArgs a0, FwdLayerArgs a1,
                                                             int tiles0) {
  __shared__ __align__(16) char smem[fwd_smem<MODE>()];
  if ((int)blockIdx.x < tiles0)
    fwd_block<MODE, TZ, A4>(a0, xcd_tile(blockIdx.x, tiles0), blockIdx.y, gridDim.y, smem);
  else if (blockIdx.y == 0)
    fwd_block<MODE, TZ, A4, true>(a1, xcd_tile(blockIdx.x - tiles0, gridDim.x - tiles0), 0, 1,
                                  smem);
}

// ---------------------------------------------------------------------------
// Grouped line-search launches: each workgroup reads its (job, local index) and
// the job's arguments through the scalar cache (uniform per workgroup, read-only
// during the launch), then runs the same body as the single-instance kernel.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T ld_uniform(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)p;
#else
  return *p;   // the host pass only parses device code
#endif
}

template <typename TZ, bool A4, class G>
__global__ __launch_bounds__(G::NT) void k_fwdlap_group(const FwdJob* __restrict__ jobs,
                                                        const GroupBlk* __restrict__ blk) {
  __shared__ __align__(16) char smem[dma_smem<G>()];
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const FwdJob j = ld_uniform(jobs + g.job);
  const int n0 = j.t0 * j.nch;
  if (g.local < n0)
    fwd_block<M_BF16, TZ, A4, false, G>(j.a0, xcd_tile(g.local % j.t0, j.t0), g.local / j.t0,
                                        j.nch, smem);
  else
    fwd_block<M_BF16, TZ, A4, true, G>(j.a1, xcd_tile(g.local - n0, j.t1), 0, 1, smem);
}


template <typename TC, typename TZ>
__global__ void k_fwdlap_finish(FwdLayerArgs a, int nch) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y + blockIdx.z * gridDim.y;
  if (c >= a.ldzo || p >= a.N) return;
  TZ* z = (TZ*)a.z;
  if (c >= a.h_out) {
    if (a.padz > 0 && c >= a.padz) return;
    for (int s = 0; s < a.S; s++)
      z[((long)s * a.N + p) * a.ldzo + c] = cvt<TZ>((c == a.h_out && s == 0) ? 1.0 : 0.0);
    return;
  }
  if (!a.has_lap) return;
  const long pc = (long)p * a.h_out + c;
  const TC t = ((const TC*)a.tab_t)[pc];
  const TC s1 = (TC)1 - t * t, s2 = (TC)-2 * t * s1;
  TC sq = 0;
  for (int k = 0; k < nch; k++) sq += ((const TC*)a.tab_sq)[(long)k * a.N * a.h_out + pc];
  const TC la = ((const TC*)a.tab_lap)[pc];
  z[((long)(a.S - 1) * a.N + p) * a.ldzo + c] = cvt<TZ>((double)(s1 * la + s2 * sq));
  if (a.sq_out) ((TC*)a.sq_out)[pc] = sq;
}

// The same with FP32 tables and 4 columns per thread (h_out and ldzo multiples
// of 4): threads [0, N h_out / 4) finish column quads of the Laplacian row, the
// rest write the bias feature and padding, one row (s, p) each.
template <typename TZ>
__device__ __forceinline__ void finish4_at(const FwdLayerArgs& a, int nch, long idx) {
  const int hq = a.h_out >> 2;
  const long nmain = a.has_lap ? (long)a.N * hq : 0;
  TZ* z = (TZ*)a.z;
  auto store4 = [](TZ* dst, const f32x4& v) {
    if constexpr (std::is_same<TZ, bf16>::value)
      *gmem((bf16x4*)dst) = __builtin_convertvector(v, bf16x4);
    else
      *gmem((f32x4*)dst) = v;
  };
  if (idx < nmain) {
    const int p = (int)(idx / hq), c = (int)(idx - (long)p * hq) * 4;
    const long pc = (long)p * a.h_out + c;
    const long plane = (long)a.N * a.h_out;
    const f32x4 t = *gmem((const f32x4*)((const float*)a.tab_t + pc));
    f32x4 sq = *gmem((const f32x4*)((const float*)a.tab_sq + pc));
    for (int k = 1; k < nch; k++) sq += *gmem((const f32x4*)((const float*)a.tab_sq + k * plane + pc));
    const f32x4 la = *gmem((const f32x4*)((const float*)a.tab_lap + pc));
    const f32x4 s1 = 1.0f - t * t, s2 = -2.0f * t * s1;
    store4(z + ((long)(a.S - 1) * a.N + p) * a.ldzo + c, s1 * la + s2 * sq);
    if (a.sq_out) *gmem((f32x4*)((float*)a.sq_out + pc)) = sq;
    return;
  }
  const long row = idx - nmain;   // s * N + p
  if (row >= (long)a.S * a.N) return;
  TZ* zr = z + row * a.ldzo;
  const long wz = a.padz > 0 ? a.padz : a.ldzo;
  for (int c = a.h_out; c < wz; c += 4) {
    f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
    if (c == a.h_out && row < a.N) v[0] = 1.0f;
    store4(zr + c, v);
  }
}
template <typename TZ>
__global__ __launch_bounds__(256) void k_fwdlap_finish4(FwdLayerArgs a, int nch) {
  finish4_at<TZ>(a, nch, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Backward layer: zbar_s = G_s W (W: h_out_next x h_in_next as rows of W^T), then
// the adjoint of the tanh rows at this layer's pre-activations:
//   gL = s1 Lbar;  g_i = s1 zbar_i + 2 [i in M] s2 d_i a Lbar;
//   g_0 = s1 zbar_0 + s2 sum_i d_i a zbar_i + (s2 La + s3 sq) Lbar   (finishing pass)
// Every chunk first recomputes the Laplacian row's cotangent Lbar.
// ---------------------------------------------------------------------------
// The same backward layer with the transposed product: a lane holds four
// consecutive neurons of one point, so every slab, table and pre-activation
// access is one 16-byte vector (all row lengths 4-aligned, FP32 rows), and each
// column kind has its own loop.  The tanh derivatives s1, s2 of each output are
// formed once.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_bwdlap_vec(BwdLayerArgs a) {
  typedef Op<MODE> O;
  typedef Geo<MODE, true> G;
  typedef Mfma<typename O::TL> MF;
  static_assert(std::is_same<typename O::TC, float>::value, "FP32 compute rows");
  __shared__ typename Mainloop<MODE, true>::Smem sm;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wp = wave >> 1, wn = wave & 1;
  const int ntc = (a.h + G::BN - 1) / G::BN;
  const int ntp = (a.N + G::BP - 1) / G::BP;
  const int t = xcd_tile(blockIdx.x, ntp * ntc);
  const int p0 = (t / ntc) * G::BP, c0 = (t % ntc) * G::BN;
  const int chunk = blockIdx.y, nch = gridDim.y;
  const int nd = a.nd;
  const int len = (nd + nch - 1) / nch;
  const int dbeg = 1 + chunk * len, dend = min(1 + nd, dbeg + len);
  const int nder = max(0, dend - dbeg);
  const int hl = a.has_lap ? 1 : 0;
  const int nsteps = hl + nder + (chunk == 0 ? 1 : 0);
  const float* pre = (const float*)a.pre;
  // output coordinates: point P(i) (lane & 15), neurons Cn(j) .. Cn(j) + 3
  int pp[G::TI], cc[G::TJ];
  bool pok[G::TI], cok[G::TJ];
#pragma unroll
  for (int i = 0; i < G::TI; i++) {
    pp[i] = p0 + wp * G::WP + i * 16 + (lane & 15);
    pok[i] = pp[i] < a.N;
  }
#pragma unroll
  for (int j = 0; j < G::TJ; j++) {
    cc[j] = c0 + wn * G::WN + j * 16 + 4 * (lane >> 4);
    cok[j] = cc[j] < a.h;
  }
  f32x4 s1[G::TI][G::TJ], s2[G::TI][G::TJ], lb[G::TI][G::TJ], sum1[G::TI][G::TJ];
#pragma unroll
  for (int i = 0; i < G::TI; i++)
#pragma unroll
    for (int j = 0; j < G::TJ; j++) {
      f32x4 tt = {0.f, 0.f, 0.f, 0.f};
      if (pok[i] && cok[j]) tt = *gmem((const f32x4*)(pre + (long)pp[i] * a.ldp + cc[j]));
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const float th = act_tanh(tt[e]);
        s1[i][j][e] = 1.f - th * th;
        s2[i][j][e] = -2.f * th * s1[i][j][e];
        lb[i][j][e] = 0.f;
        sum1[i][j][e] = 0.f;
      }
    }
  auto s_of = [=](int st) {
    if (hl && st == 0) return a.S - 1;
    const int k = st - hl;
    return k < nder ? dbeg + k : 0;
  };
  auto epi = [&](int st, int s, typename MF::acc (&acc)[G::TI][G::TJ]) __attribute__((always_inline)) {
    auto grow = [&](int i) { return (float*)a.g + ((long)s * a.N + pp[i]) * a.ldgo; };
    if (hl && st == 0) {   // Laplacian row: its cotangent, kept for the derivative rows
      const bool last = chunk == nch - 1;
#pragma unroll
      for (int i = 0; i < G::TI; i++)
#pragma unroll
        for (int j = 0; j < G::TJ; j++) {
          lb[i][j] = acc[i][j];
          if (last && pok[i] && cok[j]) {
            *gmem((f32x4*)(grow(i) + cc[j])) = s1[i][j] * acc[i][j];
            *gmem((f32x4*)((float*)a.tab_lb + (long)pp[i] * a.h + cc[j])) = acc[i][j];
          }
        }
    } else if (s >= 1 && s <= nd) {   // derivative row
      const float m2 = 2.f * wt_at(a.wts, s - 1);
#pragma unroll
      for (int i = 0; i < G::TI; i++)
#pragma unroll
        for (int j = 0; j < G::TJ; j++) {
          if (!(pok[i] && cok[j])) continue;
          const f32x4 da = *gmem((const f32x4*)(pre + ((long)s * a.N + pp[i]) * a.ldp + cc[j]));
          sum1[i][j] += da * acc[i][j];
          f32x4 o = s1[i][j] * acc[i][j];
          if (m2 != 0.f) o += m2 * s2[i][j] * da * lb[i][j];
          *gmem((f32x4*)(grow(i) + cc[j])) = o;
        }
    } else {   // value row (chunk 0)
#pragma unroll
      for (int i = 0; i < G::TI; i++)
#pragma unroll
        for (int j = 0; j < G::TJ; j++) {
          if (!(pok[i] && cok[j])) continue;
          if (hl)
            *gmem((f32x4*)((float*)a.tab_zv + (long)pp[i] * a.h + cc[j])) = acc[i][j];
          else
            *gmem((f32x4*)(grow(i) + cc[j])) = s1[i][j] * acc[i][j];
        }
    }
  };
  sloop<MODE, true, decltype(s_of), decltype(epi), true>(
      sm, (const typename O::TA*)a.gin, a.ldgi, a.N, p0, (const typename O::TB*)a.w,
      (const typename O::TB*)a.w2, a.ldw, c0, a.h, a.K, nsteps, s_of, epi);
  if (hl) {
#pragma unroll
    for (int i = 0; i < G::TI; i++)
#pragma unroll
      for (int j = 0; j < G::TJ; j++)
        if (pok[i] && cok[j])
          *gmem((f32x4*)((float*)a.tab_s1 + ((long)chunk * a.N + pp[i]) * a.h + cc[j])) =
              sum1[i][j];
  }
}

template <int MODE, typename TG>
__global__ __launch_bounds__(kThreads) void k_bwdlap(BwdLayerArgs a) {
  typedef Op<MODE> O;
  typedef Geo<MODE, true> G;
  typedef typename O::TC TC;
  typedef Mfma<typename O::TL> MF;
  __shared__ typename Mainloop<MODE, true>::Smem sm;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wp = wave >> 1, wn = wave & 1;
  const int ntc = (a.h + G::BN - 1) / G::BN;
  const int ntp = (a.N + G::BP - 1) / G::BP;
  const int t = xcd_tile(blockIdx.x, ntp * ntc);
  const int p0 = (t / ntc) * G::BP, c0 = (t % ntc) * G::BN;
  const int chunk = blockIdx.y, nch = gridDim.y;
  const int nd = a.nd;
  const int len = (nd + nch - 1) / nch;
  const int dbeg = 1 + chunk * len, dend = min(1 + nd, dbeg + len);
  const int nder = max(0, dend - dbeg);
  const int hl = a.has_lap ? 1 : 0;
  const int nsteps = hl + nder + (chunk == 0 ? 1 : 0);
  const int S = a.S;
  const TC* pre = (const TC*)a.pre;

  TC lb[G::TI][G::TJ][4], tv[G::TI][G::TJ][4], sum1[G::TI][G::TJ][4];
#pragma unroll
  for (int i = 0; i < G::TI; i++)
#pragma unroll
    for (int j = 0; j < G::TJ; j++) {
      const int c = c0 + wn * G::WN + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int p = p0 + wp * G::WP + i * 16 + MF::row(lane, e);
        TC tt = 0;
        if (p < a.N && c < a.h) tt = act_tanh(pre[(long)p * a.ldp + c]);
        tv[i][j][e] = tt;
        lb[i][j][e] = 0;
        sum1[i][j][e] = 0;
      }
    }
  // the Laplacian row first (its cotangent enters every derivative row), then
  // this chunk's derivative rows, then (chunk 0) the value row
  auto s_of = [=](int st) {
    if (hl && st == 0) return S - 1;
    const int k = st - hl;
    return k < nder ? dbeg + k : 0;
  };
  auto epi = [&](int st, int s, typename MF::acc (&acc)[G::TI][G::TJ]) {
    const bool is_lap = hl && st == 0;
    const bool is_d = !is_lap && s >= 1 && s <= nd;
    const TC m = is_d ? wt_of<TC>(a, s - 1) : (TC)0;
#pragma unroll
    for (int i = 0; i < G::TI; i++)
#pragma unroll
      for (int j = 0; j < G::TJ; j++) {
        const int c = c0 + wn * G::WN + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int p = p0 + wp * G::WP + i * 16 + MF::row(lane, e);
          const TC v = (TC)acc[i][j][e];
          const bool ok = p < a.N && c < a.h;
          const long row = (long)s * a.N + p;
          const TC tt = tv[i][j][e];
          const TC s1 = (TC)1 - tt * tt;
          if (is_lap) {
            lb[i][j][e] = v;
            if (ok && chunk == nch - 1) {
              ((TG*)a.g)[row * a.ldgo + c] = cvt<TG>((double)(s1 * v));
              ((TC*)a.tab_lb)[(long)p * a.h + c] = v;
            }
          } else if (is_d) {
            if (ok) {
              const TC da = pre[row * a.ldp + c];
              const TC s2 = (TC)-2 * tt * s1;
              sum1[i][j][e] += da * v;
              ((TG*)a.g)[row * a.ldgo + c] =
                  cvt<TG>((double)(s1 * v + (TC)2 * m * s2 * da * lb[i][j][e]));
            }
          } else if (ok) {   // value row cotangent (chunk 0)
            if (hl) ((TC*)a.tab_zv)[(long)p * a.h + c] = v;
            else ((TG*)a.g)[row * a.ldgo + c] = cvt<TG>((double)(s1 * v));
          }
        }
      }
  };
  sloop<MODE, true>(sm, (const typename O::TA*)a.gin, a.ldgi, a.N, p0, (const typename O::TB*)a.w,
              (const typename O::TB*)a.w2, a.ldw, c0, a.h, a.K, nsteps, s_of, epi);
  if (hl) {
#pragma unroll
    for (int i = 0; i < G::TI; i++)
#pragma unroll
      for (int j = 0; j < G::TJ; j++) {
        const int c = c0 + wn * G::WN + j * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int p = p0 + wp * G::WP + i * 16 + MF::row(lane, e);
          if (p < a.N && c < a.h)
            ((TC*)a.tab_s1)[((long)chunk * a.N + p) * a.h + c] = sum1[i][j][e];
        }
      }
  }
}

// value rows of g (interior) and the zero padding of g
template <typename TC, typename TG>
__global__ void k_bwdlap_finish(BwdLayerArgs a, int nch) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y + blockIdx.z * gridDim.y;
  if (c >= a.ldgo || p >= a.N) return;
  TG* g = (TG*)a.g;
  if (c >= a.h) {
    for (int s = 0; s < a.S; s++) g[((long)s * a.N + p) * a.ldgo + c] = cvt<TG>(0.0);
    return;
  }
  if (!a.has_lap) return;
  const TC* pre = (const TC*)a.pre;
  const long pc = (long)p * a.h + c;
  const TC t = act_tanh(pre[(long)p * a.ldp + c]);
  const TC s1 = (TC)1 - t * t, s2 = (TC)-2 * t * s1, s3 = (TC)-2 * s1 * ((TC)1 - (TC)3 * t * t);
  const TC la = pre[((long)(a.S - 1) * a.N + p) * a.ldp + c];
  const TC sq = ((const TC*)a.sq)[pc];
  const TC lb = ((const TC*)a.tab_lb)[pc];
  const TC zv = ((const TC*)a.tab_zv)[pc];
  TC s1sum = 0;
  for (int k = 0; k < nch; k++) s1sum += ((const TC*)a.tab_s1)[(long)k * a.N * a.h + pc];
  g[(long)p * a.ldgo + c] = cvt<TG>((double)(s1 * zv + s2 * s1sum + (s2 * la + s3 * sq) * lb));
}

// ---------------------------------------------------------------------------
// Output layer (one neuron): U[row] = z~[row] . w~  (bias in the bias column)
// ---------------------------------------------------------------------------
template <typename TZ, typename TW, typename TC>
__global__ __launch_bounds__(256) void k_last_fwd(const TZ* __restrict__ z, long ldz,
                                                  const TW* __restrict__ w, int K, long R,
                                                  TC* __restrict__ u) {
  // one wave per row: lanes stride over K
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= R) return;
  TC s = 0;
  for (int k = lane; k < K; k += 64) s += (TC)to_d(z[row * ldz + k]) * (TC)to_d(w[k]);
  s = warp_sum(s);
  if (lane == 0) u[row] = s;
}

// One line-search candidate's loss terms in one launch: each wave takes a point
// (blocks [0, nbi) the interior points, 4 per block, the rest the boundary points),
// forms its output rows as the dot products k_last_fwd forms (same order), its
// residual (interior c_t u_t + c_lap u_lap - y, boundary u - y) and the block's
// sum of squared residuals; k_ls_finalize adds the block sums of each term with
// its 1 / (2 count).
template <typename TZ, typename TW, typename TY>
__device__ __forceinline__ void ls_loss_at(const TZ* __restrict__ zi, long ldzi, int ni,
                                           int time_row, int lap_row, double c_t, double c_lap,
                                           const TY* __restrict__ yi, const TZ* __restrict__ zb,
                                           long ldzb, int nb, const TY* __restrict__ yb,
                                           const TW* __restrict__ w, int K, int nbi,
                                           double* __restrict__ partial, int bx) {
  __shared__ double red[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  auto dot = [&](const TZ* z) {
    float s = 0.f;
    for (int k = lane; k < K; k += 64) s += (float)to_d(z[k]) * (float)to_d(w[k]);
    return warp_sum(s);
  };
  const bool bnd = bx >= nbi;
  const int p = (bx - (bnd ? nbi : 0)) * 4 + wave;
  double sq = 0.0;
  if (!bnd && p < ni) {
    double v = -(double)yi[p];
    if (lap_row >= 0) v += c_lap * (double)dot(zi + ((long)lap_row * ni + p) * ldzi);
    if (time_row >= 0) v += c_t * (double)dot(zi + ((long)time_row * ni + p) * ldzi);
    sq = v * v;
  } else if (bnd && p < nb) {
    const double v = (double)dot(zb + (long)p * ldzb) - (double)yb[p];
    sq = v * v;
  }
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) partial[bx] = red[0] + red[1] + red[2] + red[3];
}
template <typename TZ, typename TW, typename TY>
__global__ __launch_bounds__(256) void k_ls_loss(const TZ* __restrict__ zi, long ldzi, int ni,
                                                 int time_row, int lap_row, double c_t,
                                                 double c_lap, const TY* __restrict__ yi,
                                                 const TZ* __restrict__ zb, long ldzb, int nb,
                                                 const TY* __restrict__ yb,
                                                 const TW* __restrict__ w, int K, int nbi,
                                                 double* __restrict__ partial) {
  ls_loss_at<TZ, TW, TY>(zi, ldzi, ni, time_row, lap_row, c_t, c_lap, yi, zb, ldzb, nb, yb, w, K,
                         nbi, partial, blockIdx.x);
}

__device__ __forceinline__ void ls_finalize_at(const double* __restrict__ partial, int nbi,
                                               int nbt, double si, double sb,
                                               double* __restrict__ loss) {
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nbt; i += 256) (i < nbi ? a : b) += partial[i];
  a = warp_sum(a);
  b = warp_sum(b);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    *loss = si * (red[0][0] + red[0][1] + red[0][2] + red[0][3]) +
            sb * (red[1][0] + red[1][1] + red[1][2] + red[1][3]);
}
__global__ __launch_bounds__(256) void k_ls_finalize(const double* __restrict__ partial, int nbi,
                                                     int nbt, double si, double sb,
                                                     double* __restrict__ loss) {
  ls_finalize_at(partial, nbi, nbt, si, sb, loss);
}

__global__ __launch_bounds__(256) void k_ls_loss_group(const LossJob* __restrict__ jobs,
                                                       const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const LossJob j = ld_uniform(jobs + g.job);
  ls_loss_at<bf16, float, float>((const bf16*)j.zi, j.ldzi, j.ni, j.time_row, j.lap_row, j.c_t,
                                 j.c_lap, j.yi, (const bf16*)j.zb, j.ldzb, j.nb, j.yb, j.w, j.K,
                                 j.nbi, j.partial, g.local);
}

__global__ __launch_bounds__(256) void k_ls_finalize_group(const LossJob* __restrict__ jobs,
                                                           int slot) {
  const LossJob j = ld_uniform(jobs + blockIdx.x);
  ls_finalize_at(j.partial, j.nbi, j.nbt, 0.5 / j.ni, 0.5 / j.nb, j.loss + slot);
}

// g of the last hidden layer from the output seeds sigma (zbar_s = sigma_s w):
// the same adjoint as k_bwdlap with an outer-product zbar.
template <typename TC, typename TSd, typename TG, typename TW>
__global__ void k_bwd_last(BwdLayerArgs a, const TSd* __restrict__ sigma, long lds,
                           const TW* __restrict__ wl) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y + blockIdx.z * gridDim.y;
  if (c >= a.ldgo || p >= a.N) return;
  TG* g = (TG*)a.g;
  if (c >= a.h) {
    for (int s = 0; s < a.S; s++) g[((long)s * a.N + p) * a.ldgo + c] = cvt<TG>(0.0);
    return;
  }
  const TC* pre = (const TC*)a.pre;
  const TC w = (TC)to_d(wl[c]);
  auto sig = [&](int s) { return (TC)to_d(sigma[((long)s * a.N + p) * lds]); };
  const TC t = act_tanh(pre[(long)p * a.ldp + c]);
  const TC s1 = (TC)1 - t * t, s2 = (TC)-2 * t * s1, s3 = (TC)-2 * s1 * ((TC)1 - (TC)3 * t * t);
  if (!a.has_lap) {
    g[(long)p * a.ldgo + c] = cvt<TG>((double)(s1 * sig(0) * w));
    return;
  }
  const TC lb = sig(a.S - 1) * w;
  const TC la = pre[((long)(a.S - 1) * a.N + p) * a.ldp + c];
  TC sum1 = 0, sq = 0;
  for (int i = 0; i < a.nd; i++) {
    const int s = 1 + i;
    const long row = (long)s * a.N + p;
    const TC da = pre[row * a.ldp + c];
    const TC zb = sig(s) * w;
    const TC m = wt_of<TC>(a, i);
    sum1 += da * zb;
    sq += m * da * da;
    g[row * a.ldgo + c] = cvt<TG>((double)(s1 * zb + (TC)2 * m * s2 * da * lb));
  }
  g[((long)(a.S - 1) * a.N + p) * a.ldgo + c] = cvt<TG>((double)(s1 * lb));
  g[(long)p * a.ldgo + c] =
      cvt<TG>((double)(s1 * sig(0) * w + s2 * sum1 + (s2 * la + s3 * sq) * lb));
}

// ---------------------------------------------------------------------------
// Input layer without products for its unit-vector rows (Section 3.1: the
// input's derivative rows are e_i and its Laplacian row is zero).
// ---------------------------------------------------------------------------
// Per neuron c: the input layer's weights of the derivative rows, stored
// transposed (wt[i * h_out + c] = W[c, i] in the product precision, W = hi [+ lo])
// so that row writers read them coalesced, and q[c] = sum_i w_i W[c, i]^2.
// A block of 256 threads takes 64 neurons and walks the inputs 64 at a time
// through an LDS tile, so that both the weight reads (along i) and the wt
// writes (along c) are coalesced; q is summed in four interleaved partial sums
// (i mod 4) added in a fixed order.
template <typename TW, typename TC>
__device__ __forceinline__ void input_q_at(const FwdLayerArgs& a, TC* __restrict__ q,
                                           TC* __restrict__ wt, int bx) {
  __shared__ TC tile[64][65];
  __shared__ TC part[4][64];
  const int t = threadIdx.x, lo = t & 63, hi = t >> 6;
  const int c0 = bx * 64;
  TC sum = 0;
  for (int i0 = 0; i0 < a.nd; i0 += 64) {
#pragma unroll 4
    for (int k = 0; k < 16; k++) {
      const int cr = hi + 4 * k, c = c0 + cr, i = i0 + lo;
      TC v = 0;
      if (c < a.h_out && i < a.nd) {
        const long e = (long)c * a.ldw + i;
        v = (TC)to_d(((const TW*)a.w)[e]) + (a.w2 ? (TC)to_d(((const TW*)a.w2)[e]) : (TC)0);
      }
      tile[cr][lo] = v;
    }
    __syncthreads();
    const int c = c0 + lo;
#pragma unroll 4
    for (int k = 0; k < 16; k++) {
      const int ir = hi + 4 * k, i = i0 + ir;
      if (c < a.h_out && i < a.nd) {
        const TC v = tile[lo][ir];
        wt[(long)i * a.h_out + c] = v;
        sum += wt_of<TC>(a, i) * v * v;
      }
    }
    __syncthreads();
  }
  part[hi][lo] = sum;
  __syncthreads();
  if (hi == 0 && c0 + lo < a.h_out)
    q[c0 + lo] = ((part[0][lo] + part[1][lo]) + part[2][lo]) + part[3][lo];
}
template <typename TW, typename TC>
__global__ __launch_bounds__(256) void k_input_q(FwdLayerArgs a, TC* __restrict__ q,
                                                 TC* __restrict__ wt) {
  input_q_at<TW, TC>(a, q, wt, blockIdx.x);
}

// The same tables when the input layer's derivative rows are general directions
// v_k (a weighted second-order operator propagated along the eigenvectors of its
// coefficient matrix): wt[k * h_out + c] = (W v_k)[c] and q[c] = sum_k w_k
// (W v_k)[c]^2, one thread per neuron, accumulated in FP64 over the d inputs.
template <typename TW, typename TC>
__global__ __launch_bounds__(256) void k_input_q_dirs(FwdLayerArgs a, TC* __restrict__ q,
                                                      TC* __restrict__ wt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.h_out) return;
  const TW* w = (const TW*)a.w + (long)c * a.ldw;
  const TW* w2 = a.w2 ? (const TW*)a.w2 + (long)c * a.ldw : nullptr;
  double sum = 0.0;
  for (int k = 0; k < a.nd; k++) {
    const double* v = a.dirs + (long)k * a.d;
    double acc = 0.0;
    for (int i = 0; i < a.d; i++) {
      const double wi = to_d(w[i]) + (w2 ? to_d(w2[i]) : 0.0);
      acc += wi * v[i];
    }
    wt[(long)k * a.h_out + c] = (TC)acc;
    sum += a.wts64[k] * acc * acc;
  }
  q[c] = (TC)sum;
}

// Eight consecutive values to z (one 16-byte store for BF16, two for FP32).  The
// BF16 rows (hundreds of MB, read back only by the next layer's product) are stored
// non-temporally: measured 12 % faster than cached stores.
template <typename TZ, typename TC>
__device__ __forceinline__ void store8(TZ* dst, const TC (&v)[8]) {
  if constexpr (std::is_same<TZ, bf16>::value) {
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; e++) o[e] = (bf16)(float)v[e];
    __builtin_nontemporal_store(o, gmem((bf16x8*)dst));
  } else if constexpr (std::is_same<TZ, float>::value) {
    const f32x4 lo = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    const f32x4 hi = {(float)v[4], (float)v[5], (float)v[6], (float)v[7]};
    *gmem((f32x4*)dst) = lo;
    *gmem((f32x4*)(dst + 4)) = hi;
  } else {
#pragma unroll
    for (int e = 0; e < 8; e++) dst[e] = cvt<TZ>((double)v[e]);
  }
}

// Eight consecutive compute-type values (two 16-byte loads for FP32).
template <typename TC>
__device__ __forceinline__ void load8(const TC* src, TC (&v)[8]) {
  if constexpr (std::is_same<TC, float>::value) {
    const f32x4 lo = *gmem((const f32x4*)src), hi = *gmem((const f32x4*)(src + 4));
#pragma unroll
    for (int e = 0; e < 4; e++) { v[e] = lo[e]; v[e + 4] = hi[e]; }
  } else {
#pragma unroll
    for (int e = 0; e < 8; e++) v[e] = src[e];
  }
}

// The 8-element arithmetic of a full chunk of derivative (or Laplacian) rows:
// z = s1 w (Laplacian row: -2 t s1 q), pre = w (0), s1 = 1 - t^2.
template <typename TC>
__device__ __forceinline__ void input_rows8(const TC (&t)[8], const TC (&w)[8], bool lap,
                                            TC (&zo)[8], TC (&po)[8]) {
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const TC s1 = (TC)1 - t[e] * t[e];
    zo[e] = lap ? (TC)-2 * t[e] * s1 * w[e] : s1 * w[e];
    po[e] = lap ? (TC)0 : w[e];
  }
}

// One 8-column chunk (row r = s N + p, columns c0 .. c0+7) of the input layer's
// rows without products: the derivative and Laplacian rows, and the padding of
// every row (value rows: only the padding; their other columns are the products').
template <typename TC, typename TZ>
__device__ __forceinline__ void input_chunk(const FwdLayerArgs& a, const TC* __restrict__ q,
                                            const TC* __restrict__ wt, long r, int s, int p,
                                            int c0) {
  const bool vec = (a.h_out & 7) == 0;
  TZ* z = (TZ*)a.z;
  const bool lap = s == a.S - 1;
  const TC* trow = (const TC*)a.tab_t + (long)p * a.h_out;
  TC zo[8], po[8];
  if (s > 0 && vec && c0 + 8 <= a.h_out) {   // full block of real columns
    TC t[8], w[8];
    load8(trow + c0, t);
    if (!lap) load8(wt + (long)(s - 1) * a.h_out + c0, w);
    else load8(q + c0, w);
    input_rows8(t, w, lap, zo, po);
    store8(z + r * a.ldzo + c0, zo);
    if (a.pre)
#pragma unroll
      for (int e = 0; e < 8; e++) ((TC*)a.pre)[r * a.ldp + c0 + e] = po[e];
    if (lap && a.sq_out)
#pragma unroll
      for (int e = 0; e < 8; e++) ((TC*)a.sq_out)[(long)p * a.h_out + c0 + e] = w[e];
    return;
  }
  // padding, a block straddling h_out, or the value row's padding
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int c = c0 + e;
    if (s == 0 && c < a.h_out) continue;   // value row: from the products
    TC zv = (c == a.h_out && s == 0) ? (TC)1 : (TC)0;
    if (c < a.h_out) {
      const TC t = trow[c];
      const TC s1 = (TC)1 - t * t;
      TC pv = 0;
      if (!lap) {
        pv = wt[(long)(s - 1) * a.h_out + c];
        zv = s1 * pv;
      } else {
        zv = (TC)-2 * t * s1 * q[c];
        if (a.sq_out) ((TC*)a.sq_out)[(long)p * a.h_out + c] = q[c];
      }
      if (a.pre) ((TC*)a.pre)[r * a.ldp + c] = pv;
    }
    z[r * a.ldzo + c] = cvt<TZ>((double)zv);
  }
}

// The rows s >= 1 and the padding of the value rows (up to padz), a thread per 8
// consecutive columns of a row, grid-stride over rows (wide rows) or over the
// rows' chunks (narrow rows).  ldzo and padz are multiples of 8; the
// vector path needs h_out to be one too (else every block takes the scalar path).
template <typename TC, typename TZ>
__device__ __forceinline__ void input_rows_at(const FwdLayerArgs& a, const TC* __restrict__ q,
                                              const TC* __restrict__ wt, long bx, long gx) {
  const long nrows = (long)a.S * a.N;
  const long wz = a.padz > 0 ? a.padz : a.ldzo;   // columns written
  auto chunk = [&](long r, int s, int p, int c0) { input_chunk<TC, TZ>(a, q, wt, r, s, p, c0); };
  // Wide rows: a wave per row, 512 columns per pass.  Narrow rows (at most 512
  // columns written, where a wave per row would leave lanes idle): the rows'
  // 8-column chunks in one flat grid-stride sequence (consecutive lanes take
  // consecutive chunks, across row ends).
  if (wz > 512) {
    const int lane = threadIdx.x & 63;
    const long nwaves = (gx * blockDim.x) >> 6;
    for (long r = (bx * blockDim.x + threadIdx.x) >> 6; r < nrows; r += nwaves) {
      const int s = (int)(r / a.N), p = (int)(r - (long)s * a.N);
      for (int c0 = lane * 8; c0 < wz; c0 += 512) chunk(r, s, p, c0);
    }
    return;
  }
  const int cpr = (int)(wz / 8);
  const long nq = nrows * cpr;
  const long i0 = bx * blockDim.x + threadIdx.x, ni = gx * blockDim.x;
  if (nq < 0x7fffffffL) {   // 32-bit index arithmetic
    for (int i = (int)i0; i < (int)nq; i += (int)ni) {
      const int r = i / cpr, s = r / a.N;
      chunk(r, s, r - s * a.N, (i - r * cpr) * 8);
    }
  } else {
    for (long i = i0; i < nq; i += ni) {
      const long r = i / cpr;
      const int s = (int)(r / a.N);
      chunk(r, s, (int)(r - (long)s * a.N), (int)(i - r * cpr) * 8);
    }
  }
}
template <typename TC, typename TZ>
__global__ __launch_bounds__(256) void k_input_rows(FwdLayerArgs a, const TC* __restrict__ q,
                                                    const TC* __restrict__ wt) {
  input_rows_at<TC, TZ>(a, q, wt, blockIdx.x, gridDim.x);
}

// The same rows point-major: workgroup (x, y) takes points [x P, x P + P) and the
// rows s of group y of gridDim.y; thread i owns items i, i + 256, ... of the
// P x (padded row / 8) grid of (point, 8-column chunk), keeps the tanh values of
// its full chunks in registers for all its rows (the row-major order reads them
// once per row), and each row's P point segments are contiguous.  Per element the
// arithmetic of input_chunk.
constexpr int kRowsPmItems = 4;   // items per thread
template <typename TC, typename TZ>
__global__ __launch_bounds__(256) void k_input_rows_pm(FwdLayerArgs a, const TC* __restrict__ q,
                                                       const TC* __restrict__ wt, int P) {
  constexpr int IT = kRowsPmItems;
  const int p0 = blockIdx.x * P;
  const int np = min(P, a.N - p0);
  if (np <= 0) return;
  const int cpr = (int)((a.padz > 0 ? a.padz : a.ldzo) / 8);
  const int items = np * cpr;
  const bool vec = (a.h_out & 7) == 0;
  const int per = (a.S + gridDim.y - 1) / gridDim.y;
  const int sb = blockIdx.y * per, se = min(a.S, sb + per);
  TC tc[IT][8];
  int col[IT], pt[IT];   // full chunk's first column (or -1) and point
#pragma unroll
  for (int k = 0; k < IT; k++) {
    const int i = threadIdx.x + 256 * k;
    const int pl = i / cpr, c0 = (i - pl * cpr) * 8;
    col[k] = (i < items && vec && c0 + 8 <= a.h_out) ? c0 : -1;
    pt[k] = p0 + pl;
    if (col[k] >= 0 && se > max(sb, 1))
      load8((const TC*)a.tab_t + (long)pt[k] * a.h_out + col[k], tc[k]);
  }
  TZ* z = (TZ*)a.z;
  for (int s = max(sb, 1); s < se; s++) {
    const bool lap = s == a.S - 1;
    const TC* wrow = lap ? q : wt + (long)(s - 1) * a.h_out;
#pragma unroll
    for (int k = 0; k < IT; k++) {
      if (col[k] < 0) continue;
      const long r = (long)s * a.N + pt[k];
      TC w[8], zo[8], po[8];
      load8(wrow + col[k], w);
      input_rows8(tc[k], w, lap, zo, po);
      store8(z + r * a.ldzo + col[k], zo);
      if (a.pre)
#pragma unroll
        for (int e = 0; e < 8; e++) ((TC*)a.pre)[r * a.ldp + col[k] + e] = po[e];
      if (lap && a.sq_out)
#pragma unroll
        for (int e = 0; e < 8; e++) ((TC*)a.sq_out)[(long)pt[k] * a.h_out + col[k] + e] = w[e];
    }
  }
  // the other chunks (padding, a chunk straddling h_out), value rows included
  for (int i = threadIdx.x; i < items; i += 256) {
    const int pl = i / cpr, c0 = (i - pl * cpr) * 8;
    if (vec && c0 + 8 <= a.h_out) continue;
#pragma unroll 1
    for (int s = sb; s < se; s++)
      input_chunk<TC, TZ>(a, q, wt, (long)s * a.N + p0 + pl, s, p0 + pl, c0);
  }
}

// Point-major when a workgroup's items cover a padded row, else row-major over g
// workgroups.  At least 2048 workgroups: rows split into groups when the points
// alone give fewer.
template <typename TC, typename TZ>
static void launch_rows_pm(const FwdLayerArgs& a, const TC* q, const TC* wt, int g,
                           hipStream_t st) {
  const int cpr = (int)((a.padz > 0 ? a.padz : a.ldzo) / 8);
  if (cpr > 256 * kRowsPmItems) {
    k_input_rows<TC, TZ><<<g, 256, 0, st>>>(a, q, wt);
    return;
  }
  const int P = std::max(1, std::min(64, 256 * kRowsPmItems / cpr));
  const int nx = (a.N + P - 1) / P;
  const int sg = std::max(1, std::min(a.S, (2048 + nx - 1) / nx));
  k_input_rows_pm<TC, TZ><<<dim3(nx, sg), 256, 0, st>>>(a, q, wt, P);
}

__global__ __launch_bounds__(256) void k_fwdlap_finish4_group(const FinJob* __restrict__ jobs,
                                                              const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const FinJob j = ld_uniform(jobs + g.job);
  finish4_at<bf16>(j.a, j.nch, (long)g.local * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_input_q_group(const InQJob* __restrict__ jobs,
                                                       const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const InQJob j = ld_uniform(jobs + g.job);
  input_q_at<bf16, float>(j.a, j.q, j.q + j.a.h_out, g.local);
}

__global__ __launch_bounds__(256) void k_input_rows_group(const InRowsJob* __restrict__ jobs,
                                                          const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const InRowsJob j = ld_uniform(jobs + g.job);
  input_rows_at<float, bf16>(j.a, j.q, j.q + j.a.h_out, g.local, j.nblk);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static dim3 pc_grid(long cols, int npts, int bs) {
  int gy = npts, gz = 1;
  while (gy > 65535) { gz *= 2; gy = (npts + gz - 1) / gz; }
  return dim3((unsigned)((cols + bs - 1) / bs), gy, gz);
}

static int compute_units() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Workgroups of `kernel` resident on one compute unit (registers and LDS permitting).
template <class F>
static int resident(F* kernel, int threads, int& cache) {
  if (cache == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1)
      n = 1;
    cache = n;
  }
  return cache;
}

// Chunks of derivative rows per layer launch.  The launch's time is simulated in
// column passes: workgroups, dispatched chunk by chunk, go to the earliest free
// of `slots` places; a chunk takes ceil(cols / ns) passes plus a start-up cost
// `ov`, where cols counts its derivative rows, the row every chunk recomputes
// (value, or the Laplacian row's cotangent) and the row that only the last
// (forward) or first (backward) chunk carries.  The chunk count with the
// shortest simulated time wins (ties: fewer chunks, less table traffic); results
// are cached per shape.
static double launch_time(int tiles, int nd, int ch, int slots, int ns, double ov,
                          bool extra_first) {
  const int len = (nd + ch - 1) / ch;
  std::priority_queue<double, std::vector<double>, std::greater<double>> q;
  for (int i = 0; i < slots; i++) q.push(0.0);
  double end = 0.0;
  for (int c = 0; c < ch; c++) {
    const int nder = std::max(0, std::min(1 + nd, 1 + (c + 1) * len) - (1 + c * len));
    const bool extra = extra_first ? c == 0 : c == ch - 1;
    const double d = (double)((1 + nder + (extra ? 1 : 0) + ns - 1) / ns) + ov;
    for (int t = 0; t < tiles; t++) {
      const double f = q.top() + d;
      q.pop();
      q.push(f);
      end = std::max(end, f);
    }
  }
  return end;
}

static int choose_chunks(int tiles, int nd, int has_lap, int slots, int ns, double ov,
                         bool extra_first) {
  if (!has_lap || nd <= 1) return 1;
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, int, bool>, int> cache;
  const auto key = std::make_tuple(tiles, nd, slots, ns, (int)(ov * 100), extra_first);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  int best = 1;
  double best_t = -1.0;
  for (int ch = 1; ch <= kMaxChunks && ch <= nd; ch++) {
    // very large launches: rounds times the longest chunk instead of the simulation
    const int len = (nd + ch - 1) / ch;
    const double t =
        (long)tiles * ch > 65536
            ? (double)(((long)tiles * ch + slots - 1) / slots) * ((len + 2 + ns - 1) / ns + ov)
            : launch_time(tiles, nd, ch, slots, ns, ov, extra_first);
    if (best_t < 0.0 || t < best_t - 1e-9) {
      best_t = t;
      best = ch;
    }
  }
  std::lock_guard<std::mutex> g(mu);
  cache[key] = best;
  return best;
}

int fwdlap_chunks(int mode, int N, int h_out, int nd, int has_lap) {
  static int occ[5] = {0, 0, 0, 0, 0};
  int per_cu = 1, ns = 1, BP = 128, BN = 128;
  switch (mode) {
    case M_BF16:
      per_cu = resident(k_fwdlap<M_BF16, bf16, true>, DGeo<M_BF16>::NT, occ[M_BF16]);
      ns = DGeo<M_BF16>::NS;
      BP = DGeo<M_BF16>::BP;
      BN = DGeo<M_BF16>::BN;
      break;
    case M_F64:
      per_cu = resident(k_fwdlap<M_F64, double>, kThreads, occ[M_F64]);
      BN = 64;
      break;
    case M_F32: per_cu = resident(k_fwdlap<M_F32, float>, kThreads, occ[M_F32]); break;
    case M_BF16X3: per_cu = resident(k_fwdlap<M_BF16X3, float>, kThreads, occ[M_BF16X3]); break;
    case M_F16: per_cu = resident(k_fwdlap<M_F16, float>, kThreads, occ[M_F16]); break;
    default: break;
  }
  const int tiles = ((N + BP - 1) / BP) * ((h_out + BN - 1) / BN);
  return choose_chunks(tiles, nd, has_lap, compute_units() * per_cu, ns, ns > 1 ? 0.3 : 1.0,
                       false);
}
int bwdlap_chunks(int mode, int N, int h, int nd, int has_lap) {
  static int occ[5] = {0, 0, 0, 0, 0};
  int per_cu = 1;
  switch (mode) {
    case M_F64: per_cu = resident(k_bwdlap<M_F64, double>, kThreads, occ[M_F64]); break;
    case M_F32: per_cu = resident(k_bwdlap<M_F32, float>, kThreads, occ[M_F32]); break;
    case M_BF16X3: per_cu = resident(k_bwdlap<M_BF16X3, float>, kThreads, occ[M_BF16X3]); break;
    case M_F16: per_cu = resident(k_bwdlap<M_F16, float>, kThreads, occ[M_F16]); break;
    default: break;
  }
  const int BP = 128, BN = 64;
  const int tiles = ((N + BP - 1) / BP) * ((h + BN - 1) / BN);
  return choose_chunks(tiles, nd, has_lap, compute_units() * per_cu, 1, 1.0, true);
}

template <int MODE, bool NARROW = false>
static dim3 tile_grid(int N, int cols, int nch) {
  typedef Geo<MODE, NARROW> G;
  return dim3(((N + G::BP - 1) / G::BP) * ((cols + G::BN - 1) / G::BN), nch);
}

template <int MODE>
static int fwd_tiles(const FwdLayerArgs& a) {
  typedef FwdGeo<MODE> G;
  return a.N > 0 ? ((a.N + G::BP - 1) / G::BP) * ((a.h_out + G::BN - 1) / G::BN) : 0;
}

template <int MODE, typename TZ, bool A4>
static void launch_fwd(const FwdLayerArgs& a0, int nch, const FwdLayerArgs* a1, hipStream_t st) {
  const int t0 = fwd_tiles<MODE>(a0);
  const int t1 = a1 ? fwd_tiles<MODE>(*a1) : 0;
  const FwdLayerArgs none{};
  k_fwdlap<MODE, TZ, A4><<<dim3(t0 + t1, nch), FwdGeo<MODE>::NT, 0, st>>>(a0, a1 ? *a1 : none, t0);
}

// padz: 0, or a multiple of 8 past the bias column and within the row
static bool pad_args_ok(const FwdLayerArgs& a) {
  return a.padz == 0 || (a.padz % 8 == 0 && a.padz > a.h_out && a.padz <= a.ldzo);
}

static bool fwd_args_ok(const FwdLayerArgs& a) {
  // the direct-to-LDS loop keeps per-point offsets in 32 bits
  return (long)a.N * a.ldz < 0x7fffffffL && (long)a.h_out * a.ldw < 0x7fffffffL &&
         pad_args_ok(a) && a.kz >= 0 && a.kz <= a.K && a.kz % 8 == 0;
}

hipError_t fwdlap_main(int mode, const FwdLayerArgs& a, int nch, hipStream_t st) {
  return fwdlap_pair(mode, a, nch, nullptr, st);
}

hipError_t fwdlap_pair(int mode, const FwdLayerArgs& a, int nch, const FwdLayerArgs* b,
                       hipStream_t st) {
  if (b && (b->N <= 0 || b->has_lap || b->value_only || b->sparse_store || b->h_out != a.h_out ||
            b->ldzo != a.ldzo || b->pre || b->w != a.w))
    return hipErrorInvalidValue;   // the second set: plain rows of the same layer
  if (a.N <= 0) return b ? fwdlap_pair(mode, *b, 1, nullptr, st) : hipSuccess;
  if (!fwd_args_ok(a) || (b && !fwd_args_ok(*b))) return hipErrorInvalidValue;
  // 4-aligned rows take the vector epilogue (table planes are 4-aligned)
  const bool a4 = (a.h_out & 3) == 0 && (a.ldzo & 3) == 0 && (!a.pre || (a.ldp & 3) == 0);
  switch (mode) {
    case M_F64: launch_fwd<M_F64, double, false>(a, nch, b, st); break;
    case M_F32:
      if (a4) launch_fwd<M_F32, float, true>(a, nch, b, st);
      else launch_fwd<M_F32, float, false>(a, nch, b, st);
      break;
    case M_BF16:
      if (a4)
        launch_fwd<M_BF16, bf16, true>(a, nch, b, st);
      else
        launch_fwd<M_BF16, bf16, false>(a, nch, b, st);
      break;
    case M_BF16X3:
      if (a4) launch_fwd<M_BF16X3, float, true>(a, nch, b, st);
      else launch_fwd<M_BF16X3, float, false>(a, nch, b, st);
      break;
    case M_F16:
      if (a4) launch_fwd<M_F16, float, true>(a, nch, b, st);
      else launch_fwd<M_F16, float, false>(a, nch, b, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fwdlap_finish(int mode, const FwdLayerArgs& a, int nch, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  if (!pad_args_ok(a)) return hipErrorInvalidValue;
  if (mode != M_F64 && (a.h_out & 3) == 0 && (a.ldzo & 3) == 0) {
    const long items = (a.has_lap ? (long)a.N * (a.h_out / 4) : 0) + (long)a.S * a.N;
    const unsigned nb = (unsigned)((items + 255) / 256);
    if (mode == M_BF16)
      k_fwdlap_finish4<bf16><<<nb, 256, 0, st>>>(a, nch);
    else
      k_fwdlap_finish4<float><<<nb, 256, 0, st>>>(a, nch);
    return hipGetLastError();
  }
  dim3 g = pc_grid(a.ldzo, a.N, 64);
  switch (mode) {
    case M_F64: k_fwdlap_finish<double, double><<<g, 64, 0, st>>>(a, nch); break;
    case M_F32: k_fwdlap_finish<float, float><<<g, 64, 0, st>>>(a, nch); break;
    case M_BF16: k_fwdlap_finish<float, bf16><<<g, 64, 0, st>>>(a, nch); break;
    case M_BF16X3:
    case M_F16: k_fwdlap_finish<float, float><<<g, 64, 0, st>>>(a, nch); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t input_layer_rows(int mode, const FwdLayerArgs& a, void* q, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  if (!a.has_lap || a.S != a.nd + 2) return hipErrorInvalidValue;
  if (a.ldzo % 8 || !pad_args_ok(a)) return hipErrorInvalidValue;
  const int nq = (a.h_out + 63) / 64;
  const int nd256 = (a.h_out + 255) / 256;
  if (a.dirs && a.d <= 0) return hipErrorInvalidValue;
  const long rows = (long)a.S * a.N;
  const int g = (int)std::min<long>(4096, (rows + 3) / 4);   // 4 rows (waves) per block
  switch (mode) {
    case M_F64: {
      double* qq = (double*)q;
      if (a.dirs)
        k_input_q_dirs<double, double><<<nd256, 256, 0, st>>>(a, qq, qq + a.h_out);
      else
        k_input_q<double, double><<<nq, 256, 0, st>>>(a, qq, qq + a.h_out);
      k_input_rows<double, double><<<g, 256, 0, st>>>(a, qq, qq + a.h_out);
      break;
    }
    case M_F32: {
      float* qq = (float*)q;
      if (a.dirs)
        k_input_q_dirs<float, float><<<nd256, 256, 0, st>>>(a, qq, qq + a.h_out);
      else
        k_input_q<float, float><<<nq, 256, 0, st>>>(a, qq, qq + a.h_out);
      k_input_rows<float, float><<<g, 256, 0, st>>>(a, qq, qq + a.h_out);
      break;
    }
    case M_BF16: {
      float* qq = (float*)q;
      if (a.dirs)
        k_input_q_dirs<bf16, float><<<nd256, 256, 0, st>>>(a, qq, qq + a.h_out);
      else
        k_input_q<bf16, float><<<nq, 256, 0, st>>>(a, qq, qq + a.h_out);
      launch_rows_pm<float, bf16>(a, qq, qq + a.h_out, g, st);
      break;
    }
    case M_BF16X3: {
      float* qq = (float*)q;
      if (a.dirs)
        k_input_q_dirs<bf16, float><<<nd256, 256, 0, st>>>(a, qq, qq + a.h_out);
      else
        k_input_q<bf16, float><<<nq, 256, 0, st>>>(a, qq, qq + a.h_out);
      k_input_rows<float, float><<<g, 256, 0, st>>>(a, qq, qq + a.h_out);
      break;
    }
    case M_F16: {
      float* qq = (float*)q;
      if (a.dirs)
        k_input_q_dirs<f16, float><<<nd256, 256, 0, st>>>(a, qq, qq + a.h_out);
      else
        k_input_q<f16, float><<<nq, 256, 0, st>>>(a, qq, qq + a.h_out);
      k_input_rows<float, float><<<g, 256, 0, st>>>(a, qq, qq + a.h_out);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bwdlap_main(int mode, const BwdLayerArgs& a, int nch, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  // FP32 rows, all row lengths 4-aligned: the vector epilogue (table planes are 4-aligned)
  const bool vec = (a.h & 3) == 0 && (a.ldp & 3) == 0 && (a.ldgo & 3) == 0;
  switch (mode) {
    case M_F64:
      k_bwdlap<M_F64, double><<<tile_grid<M_F64, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      break;
    case M_F32:
      if (vec)
        k_bwdlap_vec<M_F32><<<tile_grid<M_F32, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      else
        k_bwdlap<M_F32, float><<<tile_grid<M_F32, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      break;
    case M_BF16X3:
      if (vec)
        k_bwdlap_vec<M_BF16X3><<<tile_grid<M_BF16X3, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      else
        k_bwdlap<M_BF16X3, float><<<tile_grid<M_BF16X3, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      break;
    case M_F16:
      if (vec)
        k_bwdlap_vec<M_F16><<<tile_grid<M_F16, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      else
        k_bwdlap<M_F16, float><<<tile_grid<M_F16, true>(a.N, a.h, nch), kThreads, 0, st>>>(a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bwdlap_finish(int mode, const BwdLayerArgs& a, int nch, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  dim3 g = pc_grid(a.ldgo, a.N, 64);
  switch (mode) {
    case M_F64: k_bwdlap_finish<double, double><<<g, 64, 0, st>>>(a, nch); break;
    case M_F32: k_bwdlap_finish<float, float><<<g, 64, 0, st>>>(a, nch); break;
    case M_BF16X3:
    case M_F16: k_bwdlap_finish<float, float><<<g, 64, 0, st>>>(a, nch); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t last_fwd(int mode, const void* z, long ldz, const void* w, int K, long R, void* u,
                    hipStream_t st) {
  const int nb = (int)((R + 3) / 4);
  if (R <= 0) return hipSuccess;
  switch (mode) {
    case M_F64:
      k_last_fwd<double, double, double><<<nb, 256, 0, st>>>((const double*)z, ldz,
                                                             (const double*)w, K, R, (double*)u);
      break;
    case M_F32:
      k_last_fwd<float, float, float><<<nb, 256, 0, st>>>((const float*)z, ldz, (const float*)w,
                                                          K, R, (float*)u);
      break;
    case M_BF16:
      k_last_fwd<bf16, float, float><<<nb, 256, 0, st>>>((const bf16*)z, ldz, (const float*)w, K,
                                                         R, (float*)u);
      break;
    case M_BF16X3:
    case M_F16:
      k_last_fwd<float, float, float><<<nb, 256, 0, st>>>((const float*)z, ldz, (const float*)w,
                                                          K, R, (float*)u);
      break;
  }
  return hipGetLastError();
}

int ls_loss_blocks(int ni, int nb) { return (ni + 3) / 4 + (nb + 3) / 4; }

hipError_t ls_loss(int mode, const void* zi, long ldzi, int ni, int time_row, int lap_row,
                   double c_t, double c_lap, const void* yi, const void* zb, long ldzb, int nb,
                   const void* yb, const void* w, int K, double* partial, double* loss,
                   hipStream_t st) {
  if (mode != M_BF16 || ni <= 0 || nb <= 0) return hipErrorInvalidValue;
  const int nbi = (ni + 3) / 4, nbt = ls_loss_blocks(ni, nb);
  k_ls_loss<bf16, float, float><<<nbt, 256, 0, st>>>(
      (const bf16*)zi, ldzi, ni, time_row, lap_row, c_t, c_lap, (const float*)yi, (const bf16*)zb,
      ldzb, nb, (const float*)yb, (const float*)w, K, nbi, partial);
  k_ls_finalize<<<1, 256, 0, st>>>(partial, nbi, nbt, 0.5 / ni, 0.5 / nb, loss);
  return hipGetLastError();
}

static bool fwd_group_ok(const FwdLayerArgs& a) {
  return fwd_args_ok(a) && (a.h_out & 3) == 0 && (a.ldzo & 3) == 0 && !a.pre && !a.dirs;
}

template <class G>
static int geo_tiles(const FwdLayerArgs& a) {
  return a.N > 0 ? ((a.N + G::BP - 1) / G::BP) * ((a.h_out + G::BN - 1) / G::BN) : 0;
}

bool make_fwd_job(const FwdLayerArgs& a0, int nch, const FwdLayerArgs& a1, int geo, FwdJob* j) {
  if (a0.N <= 0 || a1.N <= 0 || a1.has_lap || a1.value_only || a1.sparse_store ||
      a1.h_out != a0.h_out || a1.ldzo != a0.ldzo || a1.w != a0.w || nch < 1 || nch > kMaxChunks ||
      geo < 0 || geo >= kFwdGeos || !fwd_group_ok(a0) || !fwd_group_ok(a1))
    return false;
  j->a0 = a0;
  j->a1 = a1;
  j->t0 = geo == 0 ? geo_tiles<DGeo<M_BF16>>(a0) : geo == 1 ? geo_tiles<DGeoW128>(a0)
                                                            : geo_tiles<DGeoW64>(a0);
  j->t1 = geo == 0 ? geo_tiles<DGeo<M_BF16>>(a1) : geo == 1 ? geo_tiles<DGeoW128>(a1)
                                                            : geo_tiles<DGeoW64>(a1);
  j->nch = nch;
  return true;
}

int fwd_geo_width(int geo) {
  return geo == 0 ? DGeo<M_BF16>::BN : geo == 1 ? DGeoW128::BN : DGeoW64::BN;
}

bool make_fin_job(const FwdLayerArgs& a, int nch, FinJob* j) {
  if (a.N <= 0 || (a.h_out & 3) != 0 || (a.ldzo & 3) != 0 || !pad_args_ok(a) || nch < 1 ||
      nch > kMaxChunks)
    return false;
  j->a = a;
  j->nch = nch;
  return true;
}

bool make_input_jobs(const FwdLayerArgs& a, void* q, int max_blocks, InQJob* jq, InRowsJob* jr) {
  if (a.N <= 0 || !a.has_lap || a.S != a.nd + 2 || a.ldzo % 8 || !pad_args_ok(a) || a.dirs ||
      max_blocks < 1)
    return false;
  jq->a = a;
  jq->q = (float*)q;
  jr->a = a;
  jr->q = (const float*)q;
  jr->nblk = (int)std::min<long>(max_blocks, ((long)a.S * a.N + 3) / 4);   // 4 rows per block
  return true;
}

int fwd_job_blocks(const FwdJob& j) { return j.t0 * j.nch + j.t1; }
int fin_job_blocks(const FinJob& j) {
  const long items = (j.a.has_lap ? (long)j.a.N * (j.a.h_out / 4) : 0) + (long)j.a.S * j.a.N;
  return (int)((items + 255) / 256);
}
int inq_job_blocks(const InQJob& j) { return (j.a.h_out + 63) / 64; }
int loss_job_blocks(const LossJob& j) { return j.nbt; }

hipError_t fwd_group(int geo, const FwdJob* jobs, const GroupBlk* blk, int nblk,
                     hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  switch (geo) {
    case 0: k_fwdlap_group<bf16, true, DGeo<M_BF16>><<<nblk, DGeo<M_BF16>::NT, 0, st>>>(jobs, blk); break;
    case 1: k_fwdlap_group<bf16, true, DGeoW128><<<nblk, DGeoW128::NT, 0, st>>>(jobs, blk); break;
    case 2: k_fwdlap_group<bf16, true, DGeoW64><<<nblk, DGeoW64::NT, 0, st>>>(jobs, blk); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t fin_group(const FinJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_fwdlap_finish4_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}
hipError_t inq_group(const InQJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_input_q_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}
hipError_t inrows_group(const InRowsJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_input_rows_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}
hipError_t loss_group(const LossJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_ls_loss_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}
hipError_t final_group(const LossJob* jobs, int njobs, int slot, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  k_ls_finalize_group<<<njobs, 256, 0, st>>>(jobs, slot);
  return hipGetLastError();
}

hipError_t bwd_last(int mode, const BwdLayerArgs& a, const void* sigma, long lds, const void* wl,
                    hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  dim3 g = pc_grid(a.ldgo, a.N, 64);
  switch (mode) {
    case M_F64:
      k_bwd_last<double, double, double, double><<<g, 64, 0, st>>>(a, (const double*)sigma, lds,
                                                                   (const double*)wl);
      break;
    case M_F32:
      k_bwd_last<float, float, float, float><<<g, 64, 0, st>>>(a, (const float*)sigma, lds,
                                                               (const float*)wl);
      break;
    case M_BF16X3:
    case M_F16:
      k_bwd_last<float, float, float, float><<<g, 64, 0, st>>>(a, (const float*)sigma, lds,
                                                               (const float*)wl);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace kp
