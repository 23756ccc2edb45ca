// Adjoint of the expected rollout cost with the noise held fixed
// (reparameterised), float and double:
//   J = (1/(K max(M,1))) sum_{k,m,t} dt q(x_{k,m,t+1}),
// and dJ/du_nom, dJ/dc_j and dJ/dD_j (every entry of D_j).
//
// Stage 1  forward sweep: 16 sub-rollouts per block, 16 lanes per sub-rollout
//          split the local models; the state is checkpointed every c steps
//          and each sub-rollout's cost sum is kept in double.
// Stage 2  reverse sweep, segment by segment from the last: the segment's
//          states and mixture moments are recomputed from its checkpoint,
//          then the state adjoint is carried backwards through the step cost,
//          explicit Euler, the sampling a = mu + sqrt(var) xi and Eq. (1):
//            ybar_j = w_j (mubar + 2 vbar (y_j - mu)),
//            qbar_j = -w_j (mubar (y_j - mu) + vbar ((y_j - mu)^2 + sigma_j^2 - var)) / 2,
//            zbar  += qbar_j (D_j + D_j^T)(z - c_j) + ybar_j b_j,
//          with mubar = abar and vbar = abar xi / (2 sqrt(var)).  Each
//          (sub-rollout, step) leaves a compact record (z, per output
//          lse, mu, var, mubar, vbar, and ubar = zbar's control part).
// Stage 3  parameter gradients: one lane per local model streams the records
//          through LDS, recomputes its weight and accumulates
//          sum qbar dl dl^T, sum qbar dl and sum ybar (dl = z - c_j); partial
//          sums per row chunk, reduced in a fixed order, then
//            dJ/dD_j = sum qbar dl dl^T,
//            dJ/dc_j = -(D_j + D_j^T) sum qbar dl - b_j sum ybar.
// Float32 problems with a matrix-core model run stages 1 and 2 on the matrix
// cores instead: the forward writes the costs and the checkpoints; then, per
// segment from the last, the segment is recomputed from its checkpoints with
// its states and moments traced, swept backwards, and its records feed the
// parameter sums (accumulated over segments) and the control gradients, so
// memory holds the checkpoints and one segment, not the whole horizon.
// Every reduction has a fixed order, so results are run-to-run identical.
// (PI^2-RH with LWPR dynamics, arXiv:1503.00330; the adjoint is not in the
// paper.)
#include <algorithm>

#include "direct.hpp"

namespace pi2rh {

constexpr int kAS = 16;                 // sub-rollouts per block
constexpr int kAL = 16;                 // lanes per sub-rollout (one DPP row)
constexpr int kAThreads = kAS * kAL;    // 256
constexpr int kParamThreads = 64;       // models per parameter-gradient block
constexpr int kParamRows = 64;          // records staged per LDS batch

template <typename Real, int DYN>
struct AdjGeo {
  using DD = DynDims<DYN>;
  static constexpr int D = DD::D, NX = DD::NX, NU = DD::NU, NO = DD::NO;
  static constexpr int RS = rec_stride<Real, D>();
  static constexpr int NP = D * (D + 1) / 2;
  static constexpr int SEGW = NX + 3 * NO;       // x_t, then (mu, var, lse) per output
  static constexpr int RW = D + 5 * NO + NU;     // z, (lse, mu, var, mubar, vbar) per output, ubar
  // matrix-core form: the trace keeps the forward's anchors per output
  // (d1, var, log2 Z, m, yref) and the records add mubar, vbar to them
  static constexpr int SEGW_M = NX + 5 * NO;
  static constexpr int RW_M = D + 7 * NO + NU;
  static constexpr int PW = NP + D + 1;          // packed sum qbar dl dl^T, sum qbar dl, sum ybar
  static constexpr int TM = tile_models<Real, D>();
};

template <typename Real>
struct AdjArgs {
  ProbDev<Real> p;
  const Real *x0, *u_nom;
  const uint32_t *iter;
  const Real *model;    // folded direct records [Ltot][RS]
  int ckpt, ncp;
  Real *ckpt_buf;       // [S][ncp][NX]
  Real *seg;            // [S][ckpt+1][SEGW]
  Real *recs;           // [S][T][RW]
  double *jsum;         // [S]
};

template <typename Real, int DYN>
struct AdjSmem {
  using G = AdjGeo<Real, DYN>;
  Real tile[G::TM * G::RS];
  Real z[kAS][G::D];
  Real x[kAS][G::NX];
  Real xbar[kAS][G::NX];
  Real xi[kAS][8];
  Real mu[kAS][G::NO], var[kAS][G::NO], lse[kAS][G::NO];
  Real mub[kAS][G::NO], vb[kAS][G::NO];
};

// Stages models j0 .. j0+nj-1 of the folded records into sm.tile.
template <typename Real, int DYN>
__device__ __forceinline__ void stage_tile(AdjSmem<Real, DYN> &sm, const Real *__restrict__ rec, int j0,
                                           int nj) {
  constexpr int RS = AdjGeo<Real, DYN>::RS;
  __syncthreads();
  for (int i = threadIdx.x; i < nj * RS; i += kAThreads) sm.tile[i] = rec[(size_t)j0 * RS + i];
  __syncthreads();
}

// Eq. (1) at sm.z[g] for all outputs; lane 0 of each group stores mu, var and
// lse = log sum_j exp(-q_j/2).  Block-synchronous.
template <typename Real, int DYN>
__device__ void adj_mixture(const ModelArgs &m, const Real *__restrict__ rec, AdjSmem<Real, DYN> &sm,
                            int g, int l) {
  using G = AdjGeo<Real, DYN>;
  Real zz[G::D];
#pragma unroll
  for (int a = 0; a < G::D; ++a) zz[a] = sm.z[g][a];
  for (int o = 0; o < G::NO; ++o) {
    MixStat<Real> st = mix_empty<Real>();
    for (int j0 = m.L_off[o]; j0 < m.L_off[o + 1]; j0 += G::TM) {
      const int nj = min(G::TM, m.L_off[o + 1] - j0);
      stage_tile(sm, rec, j0, nj);
      for (int jj = l; jj < nj; jj += kAL) {
        Real q, y;
        eval_record<Real, G::D>(sm.tile + jj * G::RS, zz, q, y);
        mix_add<false>(st, (Real)-0.5 * q, y, sm.tile[jj * G::RS + G::RS - 1]);
      }
    }
#pragma unroll
    for (int msk = 8; msk >= 1; msk >>= 1) st = mix_merge<false>(st, shfl_stat(st, msk));
    if (l == 0) {
      Real mu, v;
      mix_finish(st, &mu, &v);
      sm.mu[g][o] = mu;
      sm.var[g][o] = v;
      sm.lse[g][o] = st.m + log_(st.Z);
    }
  }
  __syncthreads();
}

// One forward step of the 16 sub-rollouts from sm.x to sm.x (lane 0 work);
// returns the step cost on lane 0 of active groups.
template <typename Real, int DYN>
__device__ Real adj_step(const AdjArgs<Real> &a, const ModelArgs &m, AdjSmem<Real, DYN> &sm, int g,
                         int l, bool active, uint32_t k, uint32_t mm, int t, uint32_t wc, uint32_t wd) {
  using G = AdjGeo<Real, DYN>;
  const ProbDev<Real> &p = a.p;
  if (l == 0) {
    if (active) {
      Real eps[4];
      normals<Real, G::NU>(p.key0, p.key1, wc, k, 0u, (uint32_t)t, eps);
#pragma unroll
      for (int i = 0; i < G::NX; ++i) sm.z[g][i] = sm.x[g][i];
#pragma unroll
      for (int i = 0; i < G::NU; ++i) sm.z[g][G::NX + i] = a.u_nom[t * G::NU + i] + p.noise_std[i] * eps[i];
      if (p.M > 0) normals<Real, G::NO>(p.key0, p.key1, wd, k, mm, (uint32_t)t, sm.xi[g]);
    } else {
#pragma unroll
      for (int i = 0; i < G::D; ++i) sm.z[g][i] = 0;
    }
  }
  __syncthreads();
  adj_mixture(m, a.model, sm, g, l);
  Real c = 0;
  if (l == 0 && active) {
    Real acc[G::NO], xs[G::NX], xn[G::NX];
#pragma unroll
    for (int o = 0; o < G::NO; ++o)
      acc[o] = p.M > 0 ? sm.mu[g][o] + sqrt_(sm.var[g][o]) * sm.xi[g][o] : sm.mu[g][o];
#pragma unroll
    for (int i = 0; i < G::NX; ++i) xs[i] = sm.x[g][i];
    euler_step<Real>(DYN, p.dt, xs, acc, &sm.z[g][G::NX], xn);  // controls sit after the state in z
#pragma unroll
    for (int i = 0; i < G::NX; ++i) sm.x[g][i] = xn[i];
    c = p.dt * state_cost<Real>(p, p.obs, xn);
  }
  return c;
}

template <typename Real, int DYN>
__global__ void __launch_bounds__(kAThreads) adj_forward_kernel(AdjArgs<Real> a, ModelArgs m) {
  using G = AdjGeo<Real, DYN>;
  __shared__ AdjSmem<Real, DYN> sm;
  const ProbDev<Real> &p = a.p;
  const int g = threadIdx.x / kAL, l = threadIdx.x % kAL;
  const int64_t S = (int64_t)p.K * p.Ms, s = (int64_t)blockIdx.x * kAS + g;
  const bool active = s < S;
  const uint32_t k = active ? (uint32_t)(s / p.Ms) : 0u, mm = active ? (uint32_t)(s % p.Ms) : 0u;
  const uint32_t it = *a.iter;
  const uint32_t wc = stream_word(kTagCtrl, p.problem_id, it), wd = stream_word(kTagDyn, p.problem_id, it);
  if (l == 0)
    for (int i = 0; i < G::NX; ++i) sm.x[g][i] = a.x0[i];
  double J = 0.0;
  for (int t = 0; t < p.T; ++t) {
    if (l == 0 && active && t % a.ckpt == 0)
      for (int i = 0; i < G::NX; ++i) a.ckpt_buf[(s * a.ncp + t / a.ckpt) * G::NX + i] = sm.x[g][i];
    J += (double)adj_step(a, m, sm, g, l, active, k, mm, t, wc, wd);
  }
  if (l == 0 && active) a.jsum[s] = J;
}

// (D + D^T)(z - c), q and y of one folded record in one traversal.
template <typename Real, int D>
__device__ __forceinline__ void eval_record_grad(const Real *__restrict__ r, const Real (&z)[D], Real &q,
                                                 Real &y, Real (&dl)[D], Real (&gq)[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    dl[a] = z[a] - r[a];
    gq[a] = 0;
  }
  const Real *th = r + D;
  q = 0;
  int idx = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Real row = 0;
#pragma unroll
    for (int b = a; b < D; ++b) {
      const Real t = th[idx++];
      row += t * dl[b];
      if (b == a) {
        gq[a] += 2 * t * dl[a];
      } else {
        gq[a] += t * dl[b];
        gq[b] += t * dl[a];
      }
    }
    q += dl[a] * row;
  }
  const Real *bb = th + D * (D + 1) / 2;
  y = bb[D];
#pragma unroll
  for (int a = 0; a < D; ++a) y += bb[a] * dl[a];
}

template <typename Real, int DYN>
__global__ void __launch_bounds__(kAThreads) adj_backward_kernel(AdjArgs<Real> a, ModelArgs m) {
  using G = AdjGeo<Real, DYN>;
  constexpr int D = G::D, NX = G::NX, NU = G::NU, NO = G::NO;
  __shared__ AdjSmem<Real, DYN> sm;
  const ProbDev<Real> &p = a.p;
  const int g = threadIdx.x / kAL, l = threadIdx.x % kAL;
  const int64_t S = (int64_t)p.K * p.Ms, s = (int64_t)blockIdx.x * kAS + g;
  const bool active = s < S;
  const uint32_t k = active ? (uint32_t)(s / p.Ms) : 0u, mm = active ? (uint32_t)(s % p.Ms) : 0u;
  const uint32_t it = *a.iter;
  const uint32_t wc = stream_word(kTagCtrl, p.problem_id, it), wd = stream_word(kTagDyn, p.problem_id, it);
  const int np = p.dyn == kDynPointMass2D ? 2 : 3;
  Real *segs = a.seg + s * (int64_t)(a.ckpt + 1) * G::SEGW;
  if (l == 0)
    for (int i = 0; i < NX; ++i) sm.xbar[g][i] = 0;
  for (int ci = a.ncp - 1; ci >= 0; --ci) {
    const int t0 = ci * a.ckpt, t1 = min(p.T, t0 + a.ckpt);
    // recompute the segment's states and mixture moments from its checkpoint
    {
      if (l == 0)
        for (int i = 0; i < NX; ++i) sm.x[g][i] = active ? a.ckpt_buf[(s * a.ncp + ci) * NX + i] : (Real)0;
      for (int t = t0; t < t1; ++t) {
        if (l == 0 && active)
          for (int i = 0; i < NX; ++i) segs[(t - t0) * G::SEGW + i] = sm.x[g][i];
        adj_step(a, m, sm, g, l, active, k, mm, t, wc, wd);
        if (l == 0 && active)
          for (int o = 0; o < NO; ++o) {
            segs[(t - t0) * G::SEGW + NX + 3 * o] = sm.mu[g][o];
            segs[(t - t0) * G::SEGW + NX + 3 * o + 1] = sm.var[g][o];
            segs[(t - t0) * G::SEGW + NX + 3 * o + 2] = sm.lse[g][o];
          }
      }
      if (l == 0 && active)
        for (int i = 0; i < NX; ++i) segs[(t1 - t0) * G::SEGW + i] = sm.x[g][i];
    }
    // reverse sweep over the segment
    for (int t = t1 - 1; t >= t0; --t) {
      if (l == 0) {
        if (active) {
          Real x1[NX], gq[NX];
          for (int i = 0; i < NX; ++i) x1[i] = segs[(t + 1 - t0) * G::SEGW + i];
          state_cost_grad<Real>(p, p.obs, x1, gq);
          for (int i = 0; i < NX; ++i) sm.xbar[g][i] += p.dt * gq[i];
          Real ab[NO];
          for (int o = 0; o < np; ++o) ab[o] = p.dt * sm.xbar[g][np + o];
          if (DYN == kDynQuad12)
            for (int o = 0; o < 3; ++o) ab[3 + o] = p.dt * sm.xbar[g][9 + o];
          Real eps[4];
          normals<Real, NU>(p.key0, p.key1, wc, k, 0u, (uint32_t)t, eps);
          if (p.M > 0) normals<Real, NO>(p.key0, p.key1, wd, k, mm, (uint32_t)t, sm.xi[g]);
          for (int i = 0; i < NX; ++i) sm.z[g][i] = segs[(t - t0) * G::SEGW + i];
          for (int i = 0; i < NU; ++i) sm.z[g][NX + i] = a.u_nom[t * NU + i] + p.noise_std[i] * eps[i];
          for (int o = 0; o < NO; ++o) {
            const Real mu = segs[(t - t0) * G::SEGW + NX + 3 * o];
            const Real v = segs[(t - t0) * G::SEGW + NX + 3 * o + 1];
            sm.mu[g][o] = mu;
            sm.var[g][o] = v;
            sm.lse[g][o] = segs[(t - t0) * G::SEGW + NX + 3 * o + 2];
            sm.mub[g][o] = ab[o];
            sm.vb[g][o] = (p.M > 0 && v > 0) ? ab[o] * sm.xi[g][o] / (2 * sqrt_(v)) : (Real)0;
          }
        } else {
          for (int i = 0; i < D; ++i) sm.z[g][i] = 0;
          for (int o = 0; o < NO; ++o) {
            sm.mu[g][o] = 0;
            sm.var[g][o] = 1;
            sm.lse[g][o] = 0;
            sm.mub[g][o] = 0;
            sm.vb[g][o] = 0;
          }
        }
      }
      __syncthreads();
      // the mixture's contribution to zbar, split over the lanes
      Real zz[D], zb[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        zz[i] = sm.z[g][i];
        zb[i] = 0;
      }
      for (int o = 0; o < NO; ++o) {
        const Real mu = sm.mu[g][o], v = sm.var[g][o], lse = sm.lse[g][o];
        const Real mub = sm.mub[g][o], vb = sm.vb[g][o];
        for (int j0 = m.L_off[o]; j0 < m.L_off[o + 1]; j0 += G::TM) {
          const int nj = min(G::TM, m.L_off[o + 1] - j0);
          stage_tile(sm, a.model, j0, nj);
          for (int jj = l; jj < nj; jj += kAL) {
            const Real *r = sm.tile + jj * G::RS;
            Real q, y, dl[D], gq[D];
            eval_record_grad<Real, D>(r, zz, q, y, dl, gq);
            const Real w = exp_((Real)-0.5 * q - lse);
            const Real e = y - mu;
            const Real ybar = w * (mub + 2 * vb * e);
            const Real qbar = (Real)-0.5 * w * (mub * e + vb * (e * e + r[G::RS - 1] - v));
            const Real *bb = r + D + D * (D + 1) / 2;
#pragma unroll
            for (int i = 0; i < D; ++i) zb[i] += qbar * gq[i] + ybar * bb[i];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int msk = 8; msk >= 1; msk >>= 1) zb[i] += __shfl_xor(zb[i], msk);
      if (l == 0 && active) {
        Real xb[NX];
        for (int i = 0; i < NX; ++i) xb[i] = sm.xbar[g][i];
        // Euler transpose: positions feed velocities, angles feed rates
        Real xp[NX];
        for (int i = 0; i < NX; ++i) xp[i] = xb[i];
        for (int i = 0; i < np; ++i) xp[np + i] += p.dt * xb[i];
        if (DYN == kDynQuad12)
          for (int i = 0; i < 3; ++i) xp[9 + i] += p.dt * xb[6 + i];
        for (int i = 0; i < NX; ++i) sm.xbar[g][i] = xp[i] + zb[i];
        Real *rec = a.recs + (s * p.T + t) * G::RW;
        for (int i = 0; i < D; ++i) rec[i] = zz[i];
        for (int o = 0; o < NO; ++o) {
          rec[D + 5 * o] = sm.lse[g][o];
          rec[D + 5 * o + 1] = sm.mu[g][o];
          rec[D + 5 * o + 2] = sm.var[g][o];
          rec[D + 5 * o + 3] = sm.mub[g][o];
          rec[D + 5 * o + 4] = sm.vb[g][o];
        }
        for (int i = 0; i < NU; ++i) rec[D + 5 * NO + i] = zb[NX + i];
      }
      __syncthreads();
    }
  }
}

// Stage 3: block (model block mb, row chunk ch); one lane per local model.
template <typename Real, int DYN>
__global__ void __launch_bounds__(kParamThreads) adj_param_kernel(ModelArgs m, const Real *__restrict__ model,
                                                                  const Real *__restrict__ recs, int64_t R,
                                                                  int nch, Real *__restrict__ gpart) {
  using G = AdjGeo<Real, DYN>;
  constexpr int D = G::D, RS = G::RS, RW = G::RW, PW = G::PW;
  __shared__ Real mrec[RS][kParamThreads];
  __shared__ Real rows[kParamRows][RW];
  const int j = blockIdx.x * kParamThreads + threadIdx.x;
  const bool valid = j < m.Ltot;
  const int ch = blockIdx.y;
  const int64_t r0 = R * ch / nch, r1 = R * (ch + 1) / nch;
  int o = 0;
  if (valid)
    while (o + 1 < m.n_out && j >= m.L_off[o + 1]) ++o;
  for (int e = 0; e < RS; ++e) mrec[e][threadIdx.x] = valid ? model[(size_t)j * RS + e] : (Real)0;
  Real acc[PW];
#pragma unroll
  for (int i = 0; i < PW; ++i) acc[i] = 0;
  Real c[D];
#pragma unroll
  for (int a = 0; a < D; ++a) c[a] = mrec[a][threadIdx.x];
  const Real s2 = mrec[RS - 1][threadIdx.x], beta0 = mrec[RS - 2][threadIdx.x];
  for (int64_t rb = r0; rb < r1; rb += kParamRows) {
    const int nr = (int)min((int64_t)kParamRows, r1 - rb);
    __syncthreads();
    for (int i = threadIdx.x; i < nr * RW; i += kParamThreads) rows[i / RW][i % RW] = recs[rb * RW + i];
    __syncthreads();
    if (!valid) continue;
    for (int rr = 0; rr < nr; ++rr) {
      Real dl[D];
#pragma unroll
      for (int a = 0; a < D; ++a) dl[a] = rows[rr][a] - c[a];
      Real q = 0, y = beta0;
      int idx = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        Real row = 0;
#pragma unroll
        for (int b = a; b < D; ++b) row += mrec[D + idx++][threadIdx.x] * dl[b];
        q += dl[a] * row;
        y += mrec[D + G::NP + a][threadIdx.x] * dl[a];
      }
      const Real *rw = &rows[rr][D + 5 * o];
      const Real lse = rw[0], mu = rw[1], v = rw[2], mub = rw[3], vb = rw[4];
      const Real w = exp_((Real)-0.5 * q - lse);
      const Real e = y - mu;
      const Real ybar = w * (mub + 2 * vb * e);
      const Real qbar = (Real)-0.5 * w * (mub * e + vb * (e * e + s2 - v));
      idx = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const Real qa = qbar * dl[a];
#pragma unroll
        for (int b = a; b < D; ++b) acc[idx++] += qa * dl[b];
      }
#pragma unroll
      for (int a = 0; a < D; ++a) acc[G::NP + a] += qbar * dl[a];
      acc[G::NP + D] += ybar;
    }
  }
  if (valid)
    for (int i = 0; i < PW; ++i) gpart[((size_t)ch * m.Ltot + j) * PW + i] = acc[i];
}

// dJ/dD_j and dJ/dc_j of one model from its centred sums (sum[0..NP) =
// sum qbar dl dl^T packed, sum[NP..NP+D) = sum qbar dl, sum[NP+D] = sum ybar,
// dl = z - c_j) and its direct record r.
template <typename Real, int D>
__device__ void param_grads_from_sums(int j, const Real *r, const double *sum, double scale, Real *gc, Real *gD) {
  constexpr int NP = D * (D + 1) / 2;
  int idx = 0;
  for (int a = 0; a < D; ++a)
    for (int b = a; b < D; ++b) {
      const double v = sum[idx++] * scale;
      gD[((size_t)j * D + a) * D + b] = (Real)v;
      gD[((size_t)j * D + b) * D + a] = (Real)v;
    }
  // (D + D^T) from the packed record: diagonal 2 theta_aa, off-diagonal theta_ab
  const Real *th = r + D;
  const Real *bb = th + NP;
  for (int a = 0; a < D; ++a) {
    double v = 0.0;
    for (int b = 0; b < D; ++b) {
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      const int pidx = lo * D - lo * (lo - 1) / 2 + (hi - lo);
      const double t = (double)th[pidx] * (a == b ? 2.0 : 1.0);
      v += t * sum[NP + b];
    }
    gc[(size_t)j * D + a] = (Real)(scale * (-v - (double)bb[a] * sum[NP + D]));
  }
}

// Stage 4a: per model, chunk partials summed in order and turned into
// dJ/dD_j and dJ/dc_j.
template <typename Real, int DYN>
__global__ void adj_param_finish_kernel(ModelArgs m, const Real *__restrict__ model, int nch,
                                        const Real *__restrict__ gpart, double scale, const double *gJ,
                                        Real *__restrict__ gc, Real *__restrict__ gD) {
  using G = AdjGeo<Real, DYN>;
  constexpr int D = G::D, RS = G::RS, PW = G::PW;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.Ltot) return;
  if (gJ) scale *= *gJ;
  double sum[PW];
  for (int i = 0; i < PW; ++i) sum[i] = 0.0;
  for (int ch = 0; ch < nch; ++ch)
    for (int i = 0; i < PW; ++i) sum[i] += (double)gpart[((size_t)ch * m.Ltot + j) * PW + i];
  param_grads_from_sums<Real, D>(j, model + (size_t)j * RS, sum, scale, gc, gD);
}

// Stage 4a, matrix-core sums: G_j = sum qbar [z z^T, z, 1] and sum ybar per
// chunk, added in chunk order in double, then centred at c_j:
//   sum qbar dl dl^T = G_zz - G_z c^T - c G_z^T + G_1 c c^T,  sum qbar dl = G_z - G_1 c.
template <int DYN>
__global__ void adj_param_mfma_finish_kernel(ModelArgs m, MfmaLayout l, const float *__restrict__ model, int nch,
                                             const float *__restrict__ gpart, int width, double scale,
                                             const double *gJ, float *__restrict__ gc, float *__restrict__ gD) {
  using G = AdjGeo<float, DYN>;
  constexpr int D = G::D, RS = G::RS, NP = G::NP, PW = G::PW;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m.Ltot) return;
  if (gJ) scale *= *gJ;
  int o = 0;
  while (o + 1 < m.n_out && j >= m.L_off[o + 1]) ++o;
  const int slot = (l.tile_off[o] + (j - m.L_off[o]) / 16) * 16 + (j - m.L_off[o]) % 16;
  double g[NP + D + 1], y = 0.0;
  for (int i = 0; i < NP + D + 1; ++i) g[i] = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    const float *src = gpart + ((size_t)ch * l.n_tiles * 16 + slot) * width;
    for (int i = 0; i < NP + D + 1; ++i) g[i] += (double)src[i];
    y += (double)src[width - 1];
  }
  const float *r = model + (size_t)j * RS;
  double c[D], gz[D];
  for (int a = 0; a < D; ++a) c[a] = (double)r[a];
  const double g1 = g[NP + D];
  for (int a = 0; a < D; ++a) gz[a] = g[NP + a];
  double sum[PW];
  int idx = 0;
  for (int a = 0; a < D; ++a)
    for (int b = a; b < D; ++b, ++idx) sum[idx] = g[idx] - gz[a] * c[b] - c[a] * gz[b] + g1 * c[a] * c[b];
  for (int a = 0; a < D; ++a) sum[NP + a] = gz[a] - g1 * c[a];
  sum[NP + D] = y;
  param_grads_from_sums<float, D>(j, r, sum, scale, gc, gD);
}

// Stage 4b: dJ/du_nom[t] = scale * sum_s ubar[s][t] (block per step, fixed tree;
// T steps of records of rw values from `recs`, ubar at offset uoff, written
// to gu[t]).
template <typename Real, int DYN>
__global__ void __launch_bounds__(256) adj_u_kernel(int64_t S, int T, const Real *__restrict__ recs, int rw,
                                                    int uoff, double scale, const double *gJ,
                                                    Real *__restrict__ gu) {
  using G = AdjGeo<Real, DYN>;
  __shared__ double red[256][G::NU];
  const int t = blockIdx.x;
  if (gJ) scale *= *gJ;
  double acc[G::NU];
  for (int i = 0; i < G::NU; ++i) acc[i] = 0.0;
  for (int64_t s = threadIdx.x; s < S; s += 256)
    for (int i = 0; i < G::NU; ++i) acc[i] += (double)recs[(s * T + t) * rw + uoff + i];
  for (int i = 0; i < G::NU; ++i) red[threadIdx.x][i] = acc[i];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int i = 0; i < G::NU; ++i) red[threadIdx.x][i] += red[threadIdx.x + w][i];
    __syncthreads();
  }
  if (threadIdx.x < G::NU) gu[t * G::NU + threadIdx.x] = (Real)(scale * red[0][threadIdx.x]);
}

// Traced forward: jsum[s] = sum_t cost[s][t] in double, one lane per sub-rollout.
__global__ void adj_jsum_kernel(int64_t S, int T, const float *__restrict__ cost, double *__restrict__ jsum) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double acc = 0.0;
  for (int t = 0; t < T; ++t) acc += (double)cost[s * T + t];
  jsum[s] = acc;
}

// Stage 4c: J = scale * sum_s jsum[s] (one block, fixed tree).
__global__ void __launch_bounds__(256) adj_j_kernel(int64_t S, const double *__restrict__ jsum, double scale,
                                                    double *__restrict__ J) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t s = threadIdx.x; s < S; s += 256) acc += jsum[s];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = scale * red[0];
}

// ------------------------------------------------------------- launcher
int adjoint_default_ckpt(int T) {
  int c = 1;
  while (c * c < T) ++c;
  return c;
}

int adjoint_param_chunks(int64_t R) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, R / 2048)); }

// record chunks of the matrix-core parameter pass over one segment of
// R records: each chunk's workgroups stream about 4096 records
static int adjoint_param_chunks_seg(int64_t R) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, R / 4096));
}

// Partial sums of the parameter pass: per chunk and model, PW values (direct)
// or adj_param_mfma_width(d) values per model slot (matrix cores; the padded
// tiles of n_out outputs add at most 16 n_out slots).
static size_t adj_gpart_bytes(int dtype, int d, int n_out, int Ltot, int64_t R, bool mfma) {
  const size_t rb = dtype == PI_F64 ? 8 : 4;
  const int pw = d * (d + 1) / 2 + d + 1;
  if (mfma)
    return align_up((size_t)adjoint_param_chunks_seg(R) * (size_t)(Ltot + 16 * n_out) * adj_param_mfma_width(d) * 4,
                    256);
  return align_up((size_t)adjoint_param_chunks(R) * Ltot * pw * rb, 256);
}

// Direct kernels: model records, checkpoints [S][ncp][NX], the segment buffer
// [S][ckpt+1][SEGW], records of every step [S][T][RW], cost sums, parameter
// partials.  Matrix-core form: model records, checkpoints, one segment's
// trace [S][ckpt+1][SEGW] and records [S][ckpt][RW], cost sums, parameter
// partials over one segment, the matrix-core tiles and reverse-sweep
// parameters, the forward costs [S][T] and the state adjoint [S][NX].
size_t adjoint_ws_bytes(int dtype, int dyn, int K, int M, int T, int Ltot, int d, int ckpt, size_t mfma_bytes) {
  const int Ms = M > 0 ? M : 1;
  const int64_t S = (int64_t)K * Ms;
  const int nx = dyn == kDynPointMass2D ? 4 : 12, nu = dyn == kDynPointMass2D ? 2 : 4,
            no = dyn == kDynPointMass2D ? 2 : 6;
  const size_t rb = dtype == PI_F64 ? 8 : 4;
  const bool mfma = mfma_bytes > 0;
  ckpt = std::max(1, std::min(ckpt, T));
  const int ncp = (T + ckpt - 1) / ckpt;
  const int segw = nx + (mfma ? 5 : 3) * no, rw = d + (mfma ? 7 : 5) * no + nu;
  const int64_t rec_steps = mfma ? ckpt : T;
  size_t b = direct_bytes(dtype, d, Ltot) + align_up((size_t)S * ncp * nx * rb, 256) +
             align_up((size_t)S * (ckpt + 1) * segw * rb, 256) + align_up((size_t)S * rec_steps * rw * rb, 256) +
             align_up((size_t)S * 8, 256) + adj_gpart_bytes(dtype, d, no, Ltot, S * rec_steps, mfma);
  if (mfma)
    b += align_up(mfma_bytes, 256) + align_up((size_t)S * T * 4, 256) + align_up((size_t)S * nx * 4, 256);
  return b;
}

template <typename Real, int DYN>
static hipError_t adjoint_t(const ProbDev<Real> &p, const ModelArgs &m, const Real *x0, const Real *u_nom,
                            const uint32_t *iter, int ckpt, const double *gJ, double *J, Real *gu, Real *gc,
                            Real *gD, void *ws, const MfmaLayout *ml, int pf, hipStream_t s) {
  using G = AdjGeo<Real, DYN>;
  const int64_t S = (int64_t)p.K * p.Ms;
  const bool mfma = ml != nullptr;
  ckpt = std::max(1, std::min(ckpt, p.T));
  const int ncp = (p.T + ckpt - 1) / ckpt;
  const int64_t rec_steps = mfma ? ckpt : p.T;
  const int64_t R = S * rec_steps;
  char *w = (char *)ws;
  AdjArgs<Real> a;
  a.p = p;
  a.x0 = x0;
  a.u_nom = u_nom;
  a.iter = iter;
  a.model = (const Real *)w;
  w += direct_bytes(sizeof(Real) == 8 ? PI_F64 : PI_F32, m.d, m.Ltot);
  a.ckpt = ckpt;
  a.ncp = ncp;
  a.ckpt_buf = (Real *)w;
  w += align_up((size_t)S * ncp * G::NX * sizeof(Real), 256);
  const int segw = mfma ? G::SEGW_M : G::SEGW, rw = mfma ? G::RW_M : G::RW;
  a.seg = (Real *)w;
  w += align_up((size_t)S * (ckpt + 1) * segw * sizeof(Real), 256);
  a.recs = (Real *)w;
  w += align_up((size_t)R * rw * sizeof(Real), 256);
  a.jsum = (double *)w;
  w += align_up((size_t)S * 8, 256);
  Real *gpart = (Real *)w;
  w += adj_gpart_bytes(sizeof(Real) == 8 ? PI_F64 : PI_F32, m.d, m.n_out, m.Ltot, R, mfma);
  hipError_t e = launch_fold_direct(sizeof(Real) == 8 ? PI_F64 : PI_F32, m, (void *)a.model, s);
  if (e != hipSuccess) return e;
  const double scale = 1.0 / (double)S;
  if constexpr (sizeof(Real) == 4) {
    if (mfma) {
      void *mbase = w;
      w += align_up(ml->bytes, 256);
      void *rfold = w;
      w += adj_rfold_bytes(*ml);
      float *cost = (float *)w;
      w += align_up((size_t)S * p.T * 4, 256);
      float *xbar = (float *)w;
      // the pieces forms' forward takes two row tiles per wave (each model
      // piece loaded serves both) once the tiles still cover the chip
      const int spw = S >= 4096 ? (pf != kPfF32 ? 32 : 16) : 8;
      e = launch_fold_mfma(PI_F32, m, *ml, mbase, s);
      if (e == hipSuccess) e = launch_adj_rfold(m, *ml, a.model, G::RS, rfold, s);
      if (e != hipSuccess) return e;
      // forward: costs (for J) and the checkpoints; a single segment is traced
      // here directly
      RolloutArgs<float> fa{p, x0, u_nom, iter, cost};
      if (ncp > 1) {
        fa.ckpt = ckpt;
        fa.ckpt_out = a.ckpt_buf;
      } else {
        fa.trace = a.seg;
        fa.trace_T = ckpt;
      }
      e = launch_rollout_mfma(fa, m, *ml, mbase, spw, 4, pf, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(adj_jsum_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, S, p.T,
                         (const float *)cost, a.jsum);
      const int nchm = adjoint_param_chunks_seg(R);
      for (int g = ncp - 1; g >= 0 && e == hipSuccess; --g) {
        const int tb = g * ckpt, te = std::min(p.T, tb + ckpt);
        if (ncp > 1) {
          // recompute the segment from its checkpoints, tracing states and moments
          RolloutArgs<float> ra{p, x0, u_nom, iter, nullptr};
          ra.t_begin = tb;
          ra.t_end = te;
          ra.ckpt = ckpt;
          ra.xstart = a.ckpt_buf;
          ra.trace = a.seg;
          ra.trace_T = ckpt;
          e = launch_rollout_mfma(ra, m, *ml, mbase, spw, 4, pf, s);
          if (e != hipSuccess) break;
        }
        e = launch_adj_reverse_mfma(p, u_nom, iter, *ml, mbase, rfold, a.seg, ckpt, tb, te, xbar, a.recs, s);
        if (e != hipSuccess) break;
        e = launch_adj_param_mfma(*ml, mbase, (const float *)a.recs, G::RW_M, S * (te - tb), nchm,
                                  (float *)gpart, g != ncp - 1, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL((adj_u_kernel<Real, DYN>), dim3(te - tb), dim3(256), 0, s, S, te - tb,
                           (const Real *)a.recs, G::RW_M, G::D + 7 * G::NO, scale, gJ, gu + (size_t)tb * G::NU);
      }
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((adj_param_mfma_finish_kernel<DYN>), dim3((m.Ltot + 63) / 64), dim3(64), 0, s, m, *ml,
                         (const float *)a.model, nchm, (const float *)gpart, adj_param_mfma_width(m.d), scale, gJ,
                         (float *)gc, (float *)gD);
      hipLaunchKernelGGL(adj_j_kernel, dim3(1), dim3(256), 0, s, S, (const double *)a.jsum, scale, J);
      return hipGetLastError();
    }
  }
  const unsigned nb = (unsigned)((S + kAS - 1) / kAS);
  const int nch = adjoint_param_chunks(R);
  hipLaunchKernelGGL((adj_forward_kernel<Real, DYN>), dim3(nb), dim3(kAThreads), 0, s, a, m);
  hipLaunchKernelGGL((adj_backward_kernel<Real, DYN>), dim3(nb), dim3(kAThreads), 0, s, a, m);
  hipLaunchKernelGGL((adj_param_kernel<Real, DYN>), dim3((m.Ltot + kParamThreads - 1) / kParamThreads, nch),
                     dim3(kParamThreads), 0, s, m, a.model, (const Real *)a.recs, R, nch, gpart);
  hipLaunchKernelGGL((adj_param_finish_kernel<Real, DYN>), dim3((m.Ltot + 63) / 64), dim3(64), 0, s, m,
                     a.model, nch, (const Real *)gpart, scale, gJ, gc, gD);
  hipLaunchKernelGGL((adj_u_kernel<Real, DYN>), dim3(p.T), dim3(256), 0, s, S, p.T, (const Real *)a.recs,
                     G::RW, G::D + 5 * G::NO, scale, gJ, gu);
  hipLaunchKernelGGL(adj_j_kernel, dim3(1), dim3(256), 0, s, S, (const double *)a.jsum, scale, J);
  return hipGetLastError();
}

hipError_t launch_adjoint(int dtype, const void *pargs, const ModelArgs &m, const void *x0, const void *u_nom,
                          const uint32_t *iter, int ckpt, const double *gJ, double *J, void *gu, void *gc,
                          void *gD, void *ws, const MfmaLayout *ml, int pf, hipStream_t s) {
  if (dtype == PI_F64) {
    const ProbDev<double> &p = *(const ProbDev<double> *)pargs;
    if (p.dyn == kDynPointMass2D)
      return adjoint_t<double, kDynPointMass2D>(p, m, (const double *)x0, (const double *)u_nom, iter, ckpt, gJ,
                                                J, (double *)gu, (double *)gc, (double *)gD, ws, nullptr, 0, s);
    return adjoint_t<double, kDynQuad12>(p, m, (const double *)x0, (const double *)u_nom, iter, ckpt, gJ, J,
                                         (double *)gu, (double *)gc, (double *)gD, ws, nullptr, 0, s);
  }
  const ProbDev<float> &p = *(const ProbDev<float> *)pargs;
  if (p.dyn == kDynPointMass2D)
    return adjoint_t<float, kDynPointMass2D>(p, m, (const float *)x0, (const float *)u_nom, iter, ckpt, gJ, J,
                                             (float *)gu, (float *)gc, (float *)gD, ws, ml, 0, s);
  return adjoint_t<float, kDynQuad12>(p, m, (const float *)x0, (const float *)u_nom, iter, ckpt, gJ, J,
                                      (float *)gu, (float *)gc, (float *)gD, ws, ml, pf, s);
}

}  // namespace pi2rh
