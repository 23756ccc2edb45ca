// Internal interfaces between the C ABI (capi.hip) and the kernel translation
// units: workspace layouts of the folded LWPR model and the host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pi2rh.h"
#include "common.hpp"

namespace pi2rh {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Raw LWPR arrays as the caller handed them (device pointers), by value.
struct ModelArgs {
  int d, n_out, R, Ltot;
  int L_off[kMaxOut + 1];
  const void *centre, *metric, *proj_u, *proj_p, *beta, *sigma2;
};

// ---- direct (VALU) folded record, one per local model ----------------------
// [c (d) | theta (d(d+1)/2, upper triangle row-major, off-diagonal entries
//  D_ab + D_ba) | b (d) | beta0 | sigma^2]:  q = sum_{a<=b} theta_ab dl_a dl_b,
// y = beta0 + b . dl with dl = z - c.  b is the PLS chain
// s_r = u_r . r_r, r_{r+1} = r_r - s_r p_r folded into one linear map.
inline int direct_stride(int d) { return d + d * (d + 1) / 2 + d + 2; }
inline size_t direct_bytes(int dtype, int d, int Ltot) {
  return align_up((size_t)Ltot * direct_stride(d) * (dtype == PI_F64 ? 8 : 4), 256);
}

// ---- MFMA (FP32) folded model ---------------------------------------------
// Models of each output are padded to tiles of 16.  For every tile the
// B-operand fragments of v_mfma_f32_16x16x4f32 for both contractions are
// stored lane-major:  W[tile][kb4][lane][4],  kblock kb = 4*kb4 + component,
// B[k][n] with k = 4*kb + lane/16 (feature), n = lane%16 (model of the tile).
// Features: kblocks [0, KQB): quadratic-form features
//   {z_a z_b (a<=b), z_a, 1, shift} with coefficients
//   {alpha theta_ab, alpha h_a, alpha kappa, 1}, h = -(D + D^T) c,
//   kappa = c^T D c, alpha = -log2(e)/2, so the product is the activation in
//   base-2 units minus a per-sample anchor (the A operand carries -anchor in
//   the shift slot);  kblocks [KQB, KQB+KYB): {z_a, 1, shift} with
//   coefficients {b_a, beta0 - b.c, 1} giving y minus a per-sample reference.
// Padded model columns get activation -1e30 (zero weight) and y = 0.
struct MfmaGeom {
  int D, NP, KQ, KQB, KY, KYB, KB, KB4;
  __host__ __device__ static MfmaGeom make(int d) {
    MfmaGeom g;
    g.D = d;
    g.NP = d * (d + 1) / 2;
    g.KQ = g.NP + d + 2;
    g.KQB = (g.KQ + 3) / 4;
    g.KY = d + 2;
    g.KYB = (g.KY + 3) / 4;
    g.KB = g.KQB + g.KYB;
    g.KB4 = (g.KB + 3) / 4;
    return g;
  }
};

// The three-piece bf16 form of the d = 16 contraction (bf16 16x16x32 matrix
// instructions): 32-feature blocks, NKQ of the quadratic-form features and
// NKY of the prediction features; per tile, block and piece (hi, mid, lo of
// the float32 value) 64 lanes x 8 bf16.
constexpr int kBfD = 16;
constexpr int kBfNKQ = (kBfD * (kBfD + 1) / 2 + kBfD + 2 + 31) / 32;   // 5
constexpr int kBfNKY = (kBfD + 2 + 31) / 32;                            // 1
constexpr int kBfNKB = kBfNKQ + kBfNKY;
constexpr size_t kBfTileU32 = (size_t)kBfNKB * 3 * 64 * 4;              // 18 KB per tile
// The two-piece fp16 form of the same blocks (fp16 16x16x32 matrix
// instructions): per tile, block and piece (hi, lo) 64 lanes x 8 fp16 of the
// values scaled per model by a power of two, and per tile 64 floats: the 16
// models' sigma^2, then the powers of two that undo the quadratic-form and
// the prediction scales, then at kHfPlain 1.0 when every scale of the tile
// is 1 (else 0.0), and zeros.
constexpr size_t kHfTileU32 = (size_t)kBfNKB * 2 * 64 * 4;              // 12 KB per tile
constexpr int kHfMeta = 64;
constexpr int kHfPlain = 48;
// Piece formats of the contraction: float32 products, or the d = 16 features
// and coefficients as three bf16 pieces (bf16 16x16x32 products), or as two
// fp16 pieces of power-of-two scaled values (fp16 16x16x32 products).
constexpr int kPfF32 = 0, kPfBf16x3 = 1, kPfF16x2 = 2;

struct MfmaLayout {
  int d, n_out, n_tiles;
  int tile_off[kMaxOut + 1];   // tile range of output o
  size_t w_floats;             // n_tiles * KB4 * 64 * 4
  size_t sig_floats;           // n_tiles * 16
  size_t wb_u32;               // the bf16 pieces (d = 16 only, else 0): n_tiles * kBfTileU32
  size_t wh_u32;               // the fp16 pieces (d = 16 only, else 0): n_tiles * kHfTileU32
  size_t hm_floats;            // their per-tile sigma^2 and scales (d = 16 only): n_tiles * kHfMeta
  size_t bytes;
};

inline MfmaLayout mfma_layout(int d, int n_out, const int *L_off) {
  MfmaLayout l;
  l.d = d;
  l.n_out = n_out;
  l.tile_off[0] = 0;
  for (int o = 0; o < n_out; ++o) l.tile_off[o + 1] = l.tile_off[o] + (L_off[o + 1] - L_off[o] + 15) / 16;
  for (int o = n_out; o < kMaxOut; ++o) l.tile_off[o + 1] = l.tile_off[n_out];
  l.n_tiles = l.tile_off[n_out];
  MfmaGeom g = MfmaGeom::make(d);
  l.w_floats = (size_t)l.n_tiles * g.KB4 * 64 * 4;
  l.sig_floats = (size_t)l.n_tiles * 16;
  l.wb_u32 = d == kBfD ? (size_t)l.n_tiles * kBfTileU32 : 0;
  l.wh_u32 = d == kBfD ? (size_t)l.n_tiles * kHfTileU32 : 0;
  l.hm_floats = d == kBfD ? (size_t)l.n_tiles * kHfMeta : 0;
  l.bytes = align_up(l.w_floats * 4, 256) + align_up(l.sig_floats * 4, 256) + align_up(l.wb_u32 * 4, 256) +
            align_up(l.wh_u32 * 4, 256) + align_up(l.hm_floats * 4, 256);
  return l;
}

// Device view of the folded MFMA model.
struct MfmaModel {
  const float4 *W;     // [n_tiles][KB4][64] float4
  const float *sig2;   // [n_tiles*16]
  const uint4 *Wb;     // [n_tiles][kBfNKB][3][64] (8 bf16 each), or null
  const uint4 *Wh;     // [n_tiles][kBfNKB][2][64] (8 fp16 each), or null
  const float *hmeta;  // [n_tiles][kHfMeta], or null
  int n_out, n_tiles;
  int tile_off[kMaxOut + 1];
};

// ---- launchers (return the first HIP error) --------------------------------
hipError_t launch_fold_direct(int dtype, const ModelArgs &m, void *rec, hipStream_t s);
hipError_t launch_fold_mfma(int dtype, const ModelArgs &m, const MfmaLayout &l, void *base,
                            hipStream_t s);

hipError_t launch_predict_direct(int dtype, const ModelArgs &m, const void *rec, const void *Z,
                                 int64_t N, void *mean, void *var, hipStream_t s);
hipError_t launch_predict_mfma(const ModelArgs &m, const MfmaLayout &l, const void *base,
                               const void *Z, int64_t N, void *mean, void *var, hipStream_t s);

template <typename Real>
struct RolloutArgs {
  ProbDev<Real> p;
  const Real *x0, *u_nom;
  const uint32_t *iter;
  Real *cost;       // [K][T] (Ms == 1) or sub-rollout costs [K][Ms][T]
  Real *trace = nullptr;  // optional [K*Ms][trace_T+1][n_x + 3 n_out]: x_t, then (mu, var, lse)
                          // of every output at step t (matrix-core kernels only)
  // Segments of the horizon (the adjoint's checkpointed forward; matrix-core
  // kernels only): steps [t_begin, t_end) (t_end < 0: T), starting from x0
  // or, with xstart, from each sub-rollout's checkpoint xstart [S][nck][n_x]
  // at slot t_begin / ckpt (nck = ceil(T / ckpt)).  With ckpt_out the state
  // before every step t with t % ckpt == 0 is stored to ckpt_out (same
  // layout).  Trace rows count from t_begin, trace_T + 1 of them per
  // sub-rollout (trace_T < 0: T).  cost may be null (nothing written).
  int t_begin = 0, t_end = -1, trace_T = -1, ckpt = 0;
  const Real *xstart = nullptr;
  Real *ckpt_out = nullptr;
};

hipError_t launch_rollout_direct(int dtype, const void *rargs, const ModelArgs &m,
                                 const void *rec, hipStream_t s);
// pf: the contraction's piece format (0 float32 products, 1 three bf16
// pieces, 2 two fp16 pieces: d = 16 quadrotor, a layout with the pieces).
hipError_t launch_rollout_mfma(const RolloutArgs<float> &ra, const ModelArgs &m,
                               const MfmaLayout &l, const void *base, int tile_samples,
                               int waves, int pf, hipStream_t s);
hipError_t launch_subcost_reduce(int dtype, const void *sub, void *cost, int K, int Ms, int T,
                                 hipStream_t s);

hipError_t launch_update(int dtype, const void *pargs, const void *cost, const uint32_t *iter,
                         void *u_nom, double *weights, void *ws, int lambda_is_double,
                         double lambda, int weighting, hipStream_t s);
size_t update_ws_bytes(int K, int T);

hipError_t launch_rh_shift(int dtype, const void *pargs, const ModelArgs &m, const void *rec,
                           void *part, void *x0, void *u_nom, const uint32_t *iter, hipStream_t s);
size_t shift_partial_bytes(const ModelArgs &m, int dtype);

// ---- batched rollouts --------------------------------------------------------
// Device descriptor of one problem of a batch and one work item (a tile of
// `spw` consecutive sub-rollouts of problem b).
struct BatchedProblem {
  ProbDev<float> p;
  const float *x0, *u_nom;
  const uint32_t *iter;
  float *cost;          // [K][T] (M <= 1) or the sub-rollout cost area in the workspace
  MfmaModel md;         // folded model inside the workspace
};
struct BatchedItem {
  int b;
  int spw;              // sub-rollouts of this item's tile (its problem's tile size)
  int64_t s_base;
};
MfmaModel mfma_model_view(const MfmaLayout &l, const void *base);
// Writes problem b's descriptor to probs[b] and its n_tiles work items
// (tiles of spw sub-rollouts, in order) to items[item_off ..], on the stream.
hipError_t launch_batched_describe(const BatchedProblem &bp, BatchedProblem *probs, BatchedItem *items, int b,
                                   int64_t item_off, int64_t n_tiles, int spw, hipStream_t s);
// max_spw: the largest tile of any item (<= 32, or 33..128 for the pieces
// forms' shared tile); waves 8 needs max_spw <= 16 or > 32; pf as above.
hipError_t launch_rollout_batched(const BatchedProblem *probs, const BatchedItem *items, int n_items,
                                  int max_spw, int waves, int pf, int grid, int *queue, hipStream_t s);
hipError_t launch_zero_int(int *p, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
// Paired-workgroup rollout (MFMA, 16 rows per pair of workgroups).
size_t pair_ws_bytes(int64_t n_groups);
int pair_grid(int64_t n_groups);
int pair_blocks_per_cu(int dyn, int waves, int pf);
hipError_t launch_rollout_pair(const RolloutArgs<float> &ra, const MfmaLayout &l, const void *base, int spw,
                               int waves, int pf, void *pair_ws, hipStream_t s);
// The device's count of paired workgroups that gave up a wait, to out[0].
hipError_t launch_read_give_ups(uint64_t *out, hipStream_t s);

// ---- adjoint -------------------------------------------------------------------
int adjoint_default_ckpt(int T);
// Adjoint parameter sums on the matrix cores (float32, d in {6, 16}): per
// record chunk and model, G = sum_r qbar Phi(z_r) (Phi = [z_a z_b, z, 1],
// padded to a multiple of 16) and sum_r ybar; adj_param_mfma_width(d) floats
// per (chunk, model slot), gpart [nch][n_tiles * 16][width].
int adj_param_mfma_width(int d);
// Adjoint reverse sweep on the matrix cores (float32): the per-model
// parameters of the second contraction are written once to `rfold`
// (adj_rfold_bytes, launch_adj_rfold); then, per segment [tb, te) of the
// horizon, one workgroup per 16 sub-rollouts sweeps t = te-1..tb over the
// segment's trace (rows counted from tb, trace_T + 1 per sub-rollout) and
// writes the segment's records [S][te - tb][d + 7 n_out + n_u].  The state
// adjoint enters from xbar_io (unless te = T) and leaves to it (unless tb = 0).
size_t adj_rfold_bytes(const MfmaLayout &l);
hipError_t launch_adj_rfold(const ModelArgs &m, const MfmaLayout &l, const void *rec, int RS, void *rfold,
                            hipStream_t s);
hipError_t launch_adj_reverse_mfma(const ProbDev<float> &p, const float *u_nom, const uint32_t *iter,
                                   const MfmaLayout &l, const void *base, const void *rfold, const float *trace,
                                   int trace_T, int tb, int te, float *xbar_io, float *recs, hipStream_t s);
// accumulate: add to gpart instead of overwriting it (later segments).
hipError_t launch_adj_param_mfma(const MfmaLayout &l, const void *base, const float *recs, int RW, int64_t R,
                                 int nch, float *gpart, bool accumulate, hipStream_t s);
// mfma_bytes > 0: float32 forward and reverse sweep on the matrix cores,
// segment by segment; 0: the direct kernels.  Both checkpoint the states
// every `ckpt` steps and recompute each segment.
size_t adjoint_ws_bytes(int dtype, int dyn, int K, int M, int T, int Ltot, int d, int ckpt, size_t mfma_bytes);
// gJ (dev, one double, nullable = 1): seed that scales every gradient.  pf:
// the piece format of the matrix-core forward and segment recomputes (the
// reverse sweep and the parameter pass contract in float32).
hipError_t launch_adjoint(int dtype, const void *pargs, const ModelArgs &m, const void *x0, const void *u_nom,
                          const uint32_t *iter, int ckpt, const double *gJ, double *J, void *gu, void *gc,
                          void *gD, void *ws, const MfmaLayout *ml, int pf, hipStream_t s);

hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t N,
                         hipStream_t s);
hipError_t launch_noise(int dtype, const void *pargs, int tag, const uint32_t *iter, int k0, int nk,
                        int m, void *out, hipStream_t s);

}  // namespace pi2rh
