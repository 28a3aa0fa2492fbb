// Fused forward-Laplacian layer products (see fwdlap.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

// chunks of derivative rows per layer launch (the finishing tables hold this many)
constexpr int kMaxChunks = 16;

// compute modes of the layer products
// M_F16: FP32 slabs rounded to FP16 on the way into LDS, weights as FP16 hi + lo,
// FP16 MFMAs with FP32 accumulation (one slab rounding per product)
enum { M_F64 = 0, M_F32 = 1, M_BF16 = 2, M_BF16X3 = 3, M_F16 = 4 };

struct FwdLayerArgs {
  const void* zin;   // input slab (s-major rows s*N + p), row length ldz, zero beyond K
  long ldz;
  const void* w;     // weights: h_out rows of length ldw (bias in column h_in)
  const void* w2;    // low parts (BF16x3) or nullptr
  long ldw;
  int K;             // h_in + 1 rounded up to 8
  int N, S, nd, has_lap, h_out;
  const float* wts;  // nd weights of the derivative rows' squares in the second-order row
  const double* wts64;  // the same weights in FP64 (read by FP64 work)
  const double* dirs;   // input-layer directions, nd rows of d (nullptr: unit vectors)
  int d;             // input dimension (directions)
  void* z;           // output slab (row length ldzo): tanh rows, bias column, zeros
  long ldzo;
  void* pre;         // optional pre-activations (row length ldp)
  long ldp;
  void* tab_t;       // N*h_out: tanh of the value row
  void* tab_sq;      // nch*N*h_out: chunk partial sums of squared derivative rows
  void* tab_lap;     // N*h_out: Laplacian-row pre-activation
  void* sq_out;      // optional N*h_out: total sum of squares (kept for the backward)
  int value_only;    // products for the value row only (the input layer, see input_layer_rows)
  int sparse_store;  // 1: z rows are stored only where needed: the value row if
  int keep_value;    //    keep_value, derivative rows s in [keep_lo, keep_hi]
  int keep_lo, keep_hi;   //    (the Laplacian row is always finished)
  int kz;            // direct-to-LDS products: input columns read (multiple of 8; the
                     //   rest of the K loop reads zeros); 0: K
  int padz;          // output columns the finishing and input-row passes write (the
                     //   bias column and zeros up to here, multiple of 8); 0: ldzo
};

struct BwdLayerArgs {
  const void* gin;   // output gradients of the next layer (rows s*N + p), row length ldgi
  long ldgi;
  const void* w;     // backward weights: h rows (this layer's width) of length ldw
  const void* w2;
  long ldw;
  int K;             // next layer's width rounded up to 8
  int N, S, nd, has_lap, h;
  const float* wts;  // nd weights (see FwdLayerArgs)
  const double* wts64;
  const void* pre;   // this layer's pre-activations (row length ldp)
  long ldp;
  const void* sq;    // N*h: sum over masked derivative rows of pre^2
  void* g;           // output gradients of this layer (row length ldgo)
  long ldgo;
  void* tab_lb;      // N*h: Laplacian-row cotangent
  void* tab_zv;      // N*h: value-row cotangent
  void* tab_s1;      // nch*N*h: chunk partials of sum_i d_i a zbar_i
};

// ---- grouped line-search launches ------------------------------------------
// One launch runs the same line-search kernel for many independent instances
// (GroupBlk, launch.h).  The jobs take the BF16 line-search path (4-aligned rows,
// unit input directions).
struct GroupBlk;
// a layer product of both point sets (fwdlap_pair): t0 tiles x nch chunks of a0,
// then t1 tiles of a1
struct FwdJob {
  FwdLayerArgs a0, a1;
  int t0, t1, nch;
};
struct FinJob {    // the finishing pass (fwdlap_finish)
  FwdLayerArgs a;
  int nch;
};
struct InQJob {    // the input layer's tables (input_layer_rows): q, then wt = q + h_out
  FwdLayerArgs a;
  float* q;
};
struct InRowsJob { // the input layer's rows without products, nblk workgroups
  FwdLayerArgs a;
  const float* q;
  int nblk;
};
struct LossJob {   // one candidate's loss (ls_loss); the finalize adds `slot` to loss
  const void* zi;
  long ldzi;
  int ni, time_row, lap_row;
  double c_t, c_lap;
  const float* yi;
  const void* zb;
  long ldzb;
  int nb;
  const float* yb;
  const float* w;
  int K, nbi, nbt;
  double* partial;
  double* loss;
};
// Job makers: false when the arguments do not take the grouped BF16 path (the
// single-instance launchers' checks, plus 4-aligned rows and unit directions).
// Tile geometries of the grouped layer product (points x neurons per workgroup):
// 0: 64 x 256 (the single-instance line search's), 1: 128 x 128, 2: 256 x 64.  An
// output element's arithmetic is the same in each.
constexpr int kFwdGeos = 3;
int fwd_geo_width(int geo);   // neurons per tile
bool make_fwd_job(const FwdLayerArgs& a0, int nch, const FwdLayerArgs& a1, int geo, FwdJob* j);
bool make_fin_job(const FwdLayerArgs& a, int nch, FinJob* j);
bool make_input_jobs(const FwdLayerArgs& a, void* q, int max_blocks, InQJob* jq, InRowsJob* jr);
// the number of workgroups of each job
int fwd_job_blocks(const FwdJob& j);
int fin_job_blocks(const FinJob& j);
int inq_job_blocks(const InQJob& j);
int loss_job_blocks(const LossJob& j);
// Grouped launches over `nblk` workgroups (blk holds nblk entries).  The
// finalize runs one workgroup per job and writes loss[slot] of each.
hipError_t fwd_group(int geo, const FwdJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);
hipError_t fin_group(const FinJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);
hipError_t inq_group(const InQJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);
hipError_t inrows_group(const InRowsJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);
hipError_t loss_group(const LossJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);
hipError_t final_group(const LossJob* jobs, int njobs, int slot, hipStream_t st);

int fwdlap_chunks(int mode, int N, int h_out, int nd, int has_lap);
hipError_t fwdlap_main(int mode, const FwdLayerArgs& a, int nch, hipStream_t st);
// One launch for two point sets of the same layer: a in nch chunks and b (or
// nullptr), plain rows without derivative or Laplacian rows (the boundary
// points), sharing a's weights and output row layout.
hipError_t fwdlap_pair(int mode, const FwdLayerArgs& a, int nch, const FwdLayerArgs* b,
                       hipStream_t st);
hipError_t fwdlap_finish(int mode, const FwdLayerArgs& a, int nch, hipStream_t st);
// The input layer's derivative and Laplacian rows without products: its input
// rows are the directions v_k (unit vectors e_k by default) and zero, so
// a_k = W v_k for every point and a_Lap = 0.  Writes z for rows s >= 1
// (z_k = s1 W v_k, z_Lap = s2 sum_k w_k (W v_k)^2),
// the bias column and padding of every row, pre and sq_out when given.  Reads t
// from tab_t (written by the value-only product).  q: scratch of (nd + 1) * h_out
// values of the compute type.
hipError_t input_layer_rows(int mode, const FwdLayerArgs& a, void* q, hipStream_t st);
int bwdlap_chunks(int mode, int N, int h, int nd, int has_lap);
hipError_t bwdlap_main(int mode, const BwdLayerArgs& a, int nch, hipStream_t st);
hipError_t bwdlap_finish(int mode, const BwdLayerArgs& a, int nch, hipStream_t st);
// output layer: u[row] = z[row] . w over K entries (bias column included)
hipError_t last_fwd(int mode, const void* z, long ldz, const void* w, int K, long R, void* u,
                    hipStream_t st);
// The loss L(theta) of one line-search candidate (BF16 slabs) from the last hidden
// layer's rows of both point sets: interior rows time_row / lap_row (< 0: absent)
// of an s-major slab of ni points, boundary rows of nb points, output weights w
// (K = h_in + 1 values, bias last); partial holds ls_loss_blocks(ni, nb) doubles.
int ls_loss_blocks(int ni, int nb);
hipError_t ls_loss(int mode, const void* zi, long ldzi, int ni, int time_row, int lap_row,
                   double c_t, double c_lap, const void* yi, const void* zb, long ldzb, int nb,
                   const void* yb, const void* w, int K, double* partial, double* loss,
                   hipStream_t st);
// gradients of the last hidden layer from output seeds sigma (row stride lds)
hipError_t bwd_last(int mode, const BwdLayerArgs& a, const void* sigma, long lds, const void* wl,
                    hipStream_t st);

}  // namespace kp
