// The POD two-grid cycle (Sec. 2.2 Alg. 2 with the POD prolongation of
// Sec. 3.3, Eq. 30) and PCG preconditioned by one cycle per iteration
// (Sec. 3.4 Alg. 3).  One thread per scalar row, 256-row workgroups, one
// grid row (blockIdx.y) per batched instance.  Every reduction is a
// deterministic two-stage tree: per-workgroup partials, then the last
// workgroup to arrive sums them in a fixed order and updates the
// instance's scalar state.  Every kernel first reads the instance's `done`
// flag and exits if it is set, so a fixed launch sequence can run past
// convergence without changing the result.
#include "common.hpp"

#include <hip/hip_ext.h>

#include <math.h>
#include <string.h>
#include <mutex>
#include <vector>

namespace pod2g {

struct Ctx {
  int n, nn, k, batch, nb, ps;   // ps: partial stride per workgroup (doubles)
  int nbn;                       // workgroups of the node-wise kernels (one thread per node)
  int N;                         // mesh elements per side
  int xwin;                      // node-wise kernels stage x[block +- xwin nodes] in LDS (0: no)
  int igroup;                    // instances per group in the node-wise block order (divides batch)
  int fuse_dir;                  // direction update folded into the outer SpMV
  int cons;                      // r^T s and p^T q finished by their consumers (else by
                                 // the producer's last workgroup)
  int fuse_upd;                  // vector update fused with the second pre-relaxation sweep
  int ptr_grp;                   // 16-row groups per wave iteration of the batched restriction
  int mixed;                     // FP32 cycle: its input is scaled by a power of two
  long long vstride;
  const int *colblk;
  const double *vals;            // FP64 K
  const void *svals;             // smoother K (FP64 or FP32)
  const void *sdinv;             // smoother D^-1
  const void *sP;                // cycle P (FP64 or FP32)
  const double *Linv;            // [batch][k][k] inverse Cholesky factor
  const float *KP32;             // [batch][k][n] FP32 K P (batched FP32 cycle, 3D) or null
  const double *KP;              // [batch][k][n] FP64 K P (setup) or null
  double omega;
  const double *f;               // [n]
  double *u, *r, *q, *s;         // [batch][n] FP64
  double *r_alt;                 // [batch][n] second residual buffer (fused update, see
                                 // k_update_sweep: the two alternate by iteration parity)
  double *p0, *p1;               // [batch][n] search directions (ping-pong)
  void *xa, *xb;                 // [batch][n] cycle vectors (smoother type)
  void *b32;                     // [batch][n] FP32 scaled residual (mixed only)
  double *part;                  // [batch][nb][ps]
  double *ec;                    // [batch][MAXK]
  InstState *st;
  double *bpart;                 // [bgrid][k][batch] partials of the batched restriction
  float *rbuf;                   // [batch][n] FP32 residuals r' of the batched restriction
  int bgrid;                     // workgroups of the batched restriction
  pod2g_slot_info *info;         // [batch] outcome of served solves
  Arrival *arr;                  // [batch][NSITE] arrival counters of the reductions
};

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int MAXB = 32;             // instances of one batched contraction
constexpr int BATCH_MFMA_MIN = 4;    // batched MFMA products from this batch size

__device__ __forceinline__ int inst_id() { return blockIdx.y; }

// Workgroup -> (node block, instance) of the node-wise kernels, whose grid
// is (nbn, batch).  Workgroups reach the 8 XCDs round-robin in linear
// order; each XCD gets one contiguous run of work items, and the items are
// ordered by instance group (igroup instances), then node block, then the
// instances of the group, so that a node block's shared column indices are
// fetched once per group and the group's gathered vectors share one L2.
struct NodeBlk {
  int blk, b;
};
__device__ __forceinline__ NodeBlk node_block(const Ctx &c) {
  const int lin = blockIdx.y * gridDim.x + blockIdx.x;
  const int w = xcd_block(lin, c.nbn * c.batch);
  const int per = c.nbn * c.igroup;
  const int grp = w / per, rem = w - grp * per;
  NodeBlk r;
  r.blk = rem / c.igroup;
  r.b = grp * c.igroup + rem % c.igroup;
  return r;
}

__device__ __forceinline__ Arrival *site(const Ctx &c, int b, int s) {
  return c.arr + (size_t)b * NSITE + s;
}

// Neighbourhood of a node block in LDS: rows of nodes [blk NT - xwin,
// blk NT + NT + xwin) of x (clamped to the instance), loaded coalesced once
// so that the block's gathers read LDS instead of cache lines of x.  In 2D
// the neighbours of node m are m +- 1, m +- N, m +- N +- 1, so xwin = N + 1
// covers them.  Returns the first staged row; every thread of the block
// must call it (it synchronises).
template <int DIM, typename T, typename XV>
__device__ __forceinline__ long long stage_x(const Ctx &c, int blk, T *xs, XV xv) {
  long long lo = (long long)blk * NT - c.xwin;
  long long hi = (long long)blk * NT + NT + c.xwin;
  lo = (lo < 0 ? 0 : lo) * DIM;
  hi = (hi > c.nn ? c.nn : hi) * DIM;
  for (long long i = lo + threadIdx.x; i < hi; i += NT) xs[i - lo] = xv((size_t)i);
  __syncthreads();
  return lo;
}

// Partial sums: slot j of instance b holds one value per workgroup,
// contiguous over workgroups.
__device__ __forceinline__ double *slot(const Ctx &c, int b, int j) {
  return c.part + ((size_t)b * c.ps + j) * c.nb;
}

// Slots of the two sums that their consumers finish themselves: r^T s from
// the end of the cycle (read by the direction update and by the vector
// update) and p^T q from the outer SpMV (read by the vector update).  The
// other reductions use slots 0 and 1 (and the restriction slots 0..k-1)
// only while these two are not live.
constexpr int SLOT_RHO = 2, SLOT_GAMMA = 3;

// Sum of m partials by every workgroup of a consumer kernel: the order of
// reduce_partials in every workgroup, so each obtains the same bits (and the
// bits the producer's last workgroup would have formed).  Every thread of
// the workgroup calls it and gets the total.
__device__ __forceinline__ double consume_partials(const double *part, int m, double *lds) {
  const double v = wave_sum(strided_sum(part, threadIdx.x, m, NT, 1));
  if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// beta of the direction update from rho_new = r^T s (Fletcher-Reeves, or
// the flexible Polak-Ribiere form with r_{k+1}^T s_k); 0 after a restart.
__device__ __forceinline__ double beta_of(const InstState *st, double trs) {
  if (st->restart) return 0.0;
  return st->beta_kind == POD2G_BETA_PR ? (trs - st->rs_prev) / st->rho : trs / st->rho;
}

// A non-positive (or non-finite) r^T s or p^T q ends the instance: every
// workgroup of the consumer skips it and one thread records it.
__device__ __forceinline__ void breakdown(InstState *st, double v) {
  st->done = 1;
  st->status = finite(v) ? POD2G_EBREAKDOWN : POD2G_ENAN;
}

// Producer side of r^T s (large grids, where every consumer workgroup
// re-reading the partials costs more than the arrival): the last workgroup
// of the cycle's final kernel forms rho and beta.
__device__ __forceinline__ void rho_tail(const Ctx &c, InstState *st, int b, int blk, double *lds,
                                         int *flag) {
  if (!arrive_last(site(c, b, CNT_B), blk, c.nbn, flag)) return;
  const double trs = reduce_partials(slot(c, b, SLOT_RHO), c.nbn, 1, lds);
  if (threadIdx.x == 0) {
    st->beta = beta_of(st, trs);
    st->restart = 0;
    st->rho = trs;
    if (!(trs > 0.0)) breakdown(st, trs);
  }
}

// a b + c with one rounding, spelled out where two kernels must agree bit
// for bit (the compiler may otherwise contract either product of a sum)
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The search direction p = s + beta p_old (beta = 0 on a restart: p = s,
// p_old not read).  One expression for the owned and the gathered entries.
__device__ __forceinline__ double pdir(double s, const double *pold, size_t i, double beta) {
  return beta == 0.0 ? s : s + beta * pold[i];
}

__device__ __forceinline__ double pow2_scale(double rr);
__device__ __forceinline__ double cycle_scale(const Ctx &c, double rr) {
  return c.mixed ? pow2_scale(rr) : 1.0;
}

__device__ __forceinline__ double pow2_scale(double rr) {
  // 2^-e with sqrt(rr) = m 2^e, m in [0.5, 1)
  if (!(rr > 0.0) || !finite(rr)) return 1.0;
  int e;
  frexp(sqrt(rr), &e);
  return ldexp(1.0, -e);
}

// ---------------------------------------------------------------- state ---
__global__ void k_state_init(InstState *st, Arrival *arr, int batch, double rtol, int maxit,
                             int beta_kind, const int *setup_status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  zero_arrivals(arr + (size_t)b * NSITE, NSITE, 0, 1);
  InstState s;
  memset(&s, 0, sizeof(s));
  s.maxit = maxit;
  s.beta_kind = beta_kind;
  s.restart = 1;
  s.scale = 1.0;
  s.tol2 = rtol * rtol;   // multiplied by ||f||^2 in k_init
  const int ss = setup_status ? setup_status[b] : 0;
  if (ss != 0) { s.done = 1; s.status = ss; }
  st[b] = s;
}

// r = f - K u; ||r||^2, ||f||^2.  Last block: tolerance and initial checks.
template <int DIM>
__global__ void __launch_bounds__(NT) k_init(Ctx c, int have_prec) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const int b = inst_id();
  InstState *st = c.st + b;
  if (st->done) return;
  const int blk = xcd_block(blockIdx.x, c.nb);
  const int row = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  double rr = 0.0, ff = 0.0;
  if (row < c.n) {
    const double kx = row_dot<DIM>(c.colblk, c.vals + (size_t)b * c.vstride, c.u + off, row,
                                   row / DIM, c.n, c.nn);
    const double fv = c.f[row];
    const double rv = fv - kx;
    c.r[off + row] = rv;
    rr = rv * rv;
    ff = fv * fv;
  }
  block_sum2(rr, ff, lds);
  if (threadIdx.x == 0) { put_partial(slot(c, b, 0) + blk, rr); put_partial(slot(c, b, 1) + blk, ff); }
  if (!arrive_last(site(c, b, CNT_A), blk, c.nb, &flag)) return;
  double trr = reduce_partials(slot(c, b, 0), c.nb, 1, lds);
  double tff = reduce_partials(slot(c, b, 1), c.nb, 1, lds);
  if (threadIdx.x == 0) {
    st->rr = trr;
    st->ff = tff;
    st->tol2 = st->tol2 * tff;
    st->scale = cycle_scale(c, trr);
    if (!finite(trr) || !finite(tff)) { st->done = 1; st->status = POD2G_ENAN; }
    else if (trr <= st->tol2) { st->done = 1; st->status = POD2G_OK; }
    if (!have_prec) st->rho = trr;
  }
}

// Cycle input b = scale * r (stored in FP32 for the mixed cycle) and, with
// write_x, the first relaxation sweep from x = 0: x = omega D^-1 b.
template <typename T>
__global__ void __launch_bounds__(NT) k_cyc_first(Ctx c, int write_x) {
  const int b = inst_id();
  if (c.st[b].done) return;
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= c.n) return;
  const size_t off = (size_t)b * c.n;
  const double sc = c.st[b].scale;
  const T bv = (T)(c.r[off + row] * sc);
  if (sizeof(T) == 4) ((float *)c.b32)[off + row] = (float)bv;
  if (write_x) ((T *)c.xa)[off + row] = (T)c.omega * ((const T *)c.sdinv)[off + row] * bv;
}

template <typename T>
__device__ __forceinline__ const T *cycle_rhs(const Ctx &c, size_t off) {
  return sizeof(T) == 8 ? (const T *)(c.r + off) : (const T *)c.b32 + off;
}

// x_out = x_in + omega D^-1 (b - K x_in), one thread per node (its DIM
// rows).  With FINAL the result is the preconditioned residual
// s = x_out / scale (FP64) and the block also writes its partial of r^T s
// (finished by the consumers: k_pdir or k_spmv_pq, and k_update; or, with
// c.cons unset, by the last workgroup here, which forms rho and beta).
template <int DIM, typename T, bool FINAL>
__global__ void __launch_bounds__(NT) k_sweep(Ctx c, const T *__restrict__ xin, T *__restrict__ xout,
                                              int want_dot) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const NodeBlk nbk = node_block(c);
  const int b = nbk.b, blk = nbk.blk;
  InstState *st = c.st ? c.st + b : nullptr;   // null: standalone sweeps
  // One instance: a finished instance is skipped at its first store, so the
  // state load is in flight with the gathers instead of ahead of them (the
  // few launches after convergence cost little).  Several instances (a batch,
  // served slots, most of them possibly finished or free): skip at once.
  if (c.batch > 1 && st && st->done) return;
  const int done = st ? st->done : 0;
  const int node = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  const T *xb = xin + off;
  extern __shared__ double xlds_dyn[];
  T *xs = (T *)xlds_dyn;
  const long long xlo = c.xwin ? stage_x<DIM, T>(c, blk, xs, [xb](size_t i) { return xb[i]; }) : 0;
  double rs = 0.0;
  if (node < c.nn) {
    const T *vals = (const T *)c.svals + (size_t)b * c.vstride;
    T kx[DIM];
    if (c.xwin)
      node_dot<DIM>(c.colblk, vals, [xs, xlo](size_t i) { return xs[i - xlo]; }, node, c.n, c.nn, kx);
    else
      node_dot<DIM>(c.colblk, vals, [xb](size_t i) { return xb[i]; }, node, c.n, c.nn, kx);
    const size_t r0 = off + (size_t)node * DIM;
    const T *rhs = cycle_rhs<T>(c, off) + (size_t)node * DIM;
    const T *dv = (const T *)c.sdinv + r0;
    if (done) return;
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
      const T xv = fma_t((T)c.omega * dv[r], rhs[r] - kx[r], xin[r0 + r]);
      if (FINAL) {
        const double sv = (double)xv / st->scale;
        c.s[r0 + r] = sv;
        rs += c.r[r0 + r] * sv;
      } else {
        xout[r0 + r] = xv;
      }
    }
  }
  if (!FINAL || !want_dot || done) return;
  double dummy = 0.0;
  block_sum2(rs, dummy, lds);
  if (threadIdx.x == 0) put_partial(slot(c, b, SLOT_RHO) + blk, rs);
  if (!c.cons) rho_tail(c, st, b, blk, lds, &flag);
}

// Residual after pre-relaxation and restriction: r' = b - K x,
// r_c = P^T r'; the last block solves L L^T e_c = r_c (FP64).
template <int DIM, typename T, bool XZERO>
__global__ void __launch_bounds__(NT) k_restrict(Ctx c, const T *__restrict__ x,
                                                 T *__restrict__ rsave) {
  __shared__ double lds[2 * NWAVE];
  __shared__ double rsh[NT];
  __shared__ double rc[MAXK];
  __shared__ int flag;
  const int b = inst_id();
  InstState *st = c.st + b;
  if (c.batch > 1 && st->done) return;
  const int done = st->done;   // one instance: checked at the first store (see k_sweep)
  const int blk = xcd_block(blockIdx.x, c.nb);
  const int row = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  T rv = T(0);
  if (row < c.n) {
    const T bv = cycle_rhs<T>(c, off)[row];
    if (XZERO) {
      rv = bv;
    } else {
      const T *vals = (const T *)c.svals + (size_t)b * c.vstride;
      rv = bv - row_dot<DIM>(c.colblk, vals, x + off, row, row / DIM, c.n, c.nn);
    }
  }
  if (done) return;
  if (row < c.n && rsave) rsave[off + row] = rv;   // r' for the first post-sweep (see k_prolong)
  rsh[threadIdx.x] = (double)rv;
  __syncthreads();
  // wave w reduces columns j = w, w + 4, ...; lane l covers rows l + 64 m
  const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  const T *P = (const T *)c.sP;
  const int row0 = blk * NT;
  // this wave's columns j = w + NWAVE q, four at a time so that their P
  // loads are in flight together
  const int ncol = (c.k - w + NWAVE - 1) / NWAVE;
  for (int q0 = 0; q0 < ncol; q0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // unguarded loads (a guarded load is a branch, and the compiler then
    // waits for each before the next): rows past n read row n - 1 and meet
    // r' = 0, columns past this wave's share read column k - 1 and are
    // discarded
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const int j = w + (q0 + cc) * NWAVE;
      const T *Pj = P + (size_t)(j < c.k ? j : c.k - 1) * c.n;
#pragma unroll
      for (int m = 0; m < NT / WAVE; ++m) {
        const int rr = row0 + lane + m * WAVE;
        acc[cc] += (double)Pj[rr < c.n ? rr : c.n - 1] * rsh[lane + m * WAVE];
      }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) acc[cc] = wave_sum(acc[cc]);
    if (lane == 0) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
        if (q0 + cc < ncol) rc[w + (q0 + cc) * NWAVE] = acc[cc];
    }
  }
  __syncthreads();
  if (threadIdx.x < c.k) put_partial(slot(c, b, threadIdx.x) + blk, rc[threadIdx.x]);
  if (!arrive_last(site(c, b, CNT_C), blk, c.nb, &flag)) return;
  const int k = c.k;
  // the inverse factor into LDS (dynamic, k x k), its loads in flight with
  // those of the partials
  extern __shared__ double Ls[];
  const double *Li = c.Linv + (size_t)b * k * k;
  for (int t0 = 0; t0 < k * k; t0 += 4 * NT) {
    double lv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * NT + threadIdx.x;
      lv[u] = Li[t < k * k ? t : k * k - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * NT + threadIdx.x;
      if (t < k * k) Ls[t] = lv[u];
    }
  }
  // r_c: tpc threads per column, each summing a strided share of the
  // column's partials, then the shares in order
  const int tpc = NT / k;
  if (threadIdx.x < k * tpc)
    rsh[threadIdx.x] = strided_sum_wide(slot(c, b, threadIdx.x / tpc), threadIdx.x % tpc, c.nb,
                                        tpc, 1);
  __syncthreads();
  if (threadIdx.x < k) {
    double v = 0.0;
    for (int q = 0; q < tpc; ++q) v += rsh[threadIdx.x * tpc + q];
    rc[threadIdx.x] = v;
  }
  __syncthreads();
  // coarse solve L L^T e_c = r_c as e_c = Linv^T (Linv r_c)
  double y = 0.0;
  if (threadIdx.x < k) {
    const int i = threadIdx.x;
    for (int j = 0; j <= i; ++j) y += Ls[i * k + j] * rc[j];
  }
  __syncthreads();
  if (threadIdx.x < k) rsh[threadIdx.x] = y;
  __syncthreads();
  if (threadIdx.x < k) {
    const int i = threadIdx.x;
    double e = 0.0;
    for (int j = i; j < k; ++j) e += Ls[j * k + i] * rsh[j];
    c.ec[(size_t)b * MAXK + i] = e;
  }
}

// Residual after pre-relaxation for the batched restriction:
// r'_b = b_b - K_b x_b stored in FP32 (one thread per row, one grid row per
// instance, no reduction).
template <int DIM>
__global__ void __launch_bounds__(NT) k_resid32(Ctx c, const float *__restrict__ x) {
  const NodeBlk nbk = node_block(c);
  const int b = nbk.b;
  if (c.st[b].done) return;
  const int node = nbk.blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  const float *xb = x + off;
  extern __shared__ double xlds_dyn[];
  float *xs = (float *)xlds_dyn;
  const long long xlo =
      c.xwin ? stage_x<DIM, float>(c, nbk.blk, xs, [xb](size_t i) { return xb[i]; }) : 0;
  if (node >= c.nn) return;
  const float *vals = (const float *)c.svals + (size_t)b * c.vstride;
  float kx[DIM];
  if (c.xwin)
    node_dot<DIM>(c.colblk, vals, [xs, xlo](size_t i) { return xs[i - xlo]; }, node, c.n, c.nn, kx);
  else
    node_dot<DIM>(c.colblk, vals, [xb](size_t i) { return xb[i]; }, node, c.n, c.nn, kx);
  const size_t r0 = off + (size_t)node * DIM;
#pragma unroll
  for (int r = 0; r < DIM; ++r) c.rbuf[r0 + r] = ((const float *)c.b32)[r0 + r] - kx[r];
}

// Prolongation and correction: x_out = x_in + P e_c.  With rp (the
// restricted residual r') and kp (the instance's K P) it also applies the
// first post-relaxation sweep from b - K (x + P e_c) = r' - (K P) e_c.
template <typename T>
__global__ void __launch_bounds__(NT) k_prolong(Ctx c, const T *__restrict__ xin, T *__restrict__ xout,
                                                const T *__restrict__ rp, const T *__restrict__ kp) {
  constexpr int PC = 16;   // basis (and K P) loads in flight together
  const int b = inst_id();
  if (c.batch > 1 && c.st[b].done) return;
  const int done = c.st[b].done;   // one instance: checked at the store (see k_sweep)
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= c.n) return;
  const size_t off = (size_t)b * c.n;
  const T *P = (const T *)c.sP;
  const double *ec = c.ec + (size_t)b * MAXK;   // the same for every lane
  T acc = xin ? xin[off + row] : T(0);
  T d = rp ? rp[off + row] : T(0);
  const T *kpb = rp ? kp + (size_t)b * c.k * c.n + row : nullptr;
  for (int j0 = 0; j0 < c.k; j0 += PC) {
    T pv[PC], kv[PC];
#pragma unroll
    for (int u = 0; u < PC; ++u) {
      pv[u] = j0 + u < c.k ? P[(size_t)(j0 + u) * c.n + row] : T(0);
      kv[u] = (kpb && j0 + u < c.k) ? kpb[(size_t)(j0 + u) * c.n] : T(0);
    }
#pragma unroll
    for (int u = 0; u < PC; ++u) {
      const T eu = j0 + u < c.k ? (T)ec[j0 + u] : T(0);
      acc += pv[u] * eu;
      d -= kv[u] * eu;
    }
  }
  if (done) return;
  if (rp) acc += (T)c.omega * ((const T *)c.sdinv)[off + row] * d;
  xout[off + row] = acc;
}

// s = x / scale with r^T s (used when the cycle ends without a sweep),
// one thread per node; the partials of r^T s go where k_sweep puts them.
template <int DIM, typename T>
__global__ void __launch_bounds__(NT) k_finalize(Ctx c, const T *__restrict__ x, int want_dot) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const NodeBlk nbk = node_block(c);
  const int b = nbk.b, blk = nbk.blk;
  InstState *st = c.st + b;
  if (st->done) return;
  const int node = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  double rs = 0.0;
  if (node < c.nn) {
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
      const size_t row = off + (size_t)node * DIM + r;
      const double sv = x ? (double)x[row] / st->scale : 0.0;
      c.s[row] = sv;
      rs += c.r[row] * sv;
    }
  }
  if (!want_dot) return;
  double dummy = 0.0;
  block_sum2(rs, dummy, lds);
  if (threadIdx.x == 0) put_partial(slot(c, b, SLOT_RHO) + blk, rs);
  if (!c.cons) rho_tail(c, st, b, blk, lds, &flag);
}

// q = K p and the partials of p^T q, one thread per node; k_update
// finishes the sum (c.cons) or the last workgroup here forms alpha.  With
// FUSED the direction p = s + beta p_old is formed here (gathered where K
// needs it, the owned rows written to pnew), beta from the cycle's r^T s
// partials when cons and c.cons are set (else the beta in the state);
// otherwise k_pdir formed it already.  Workgroup 0 sets the input scale of
// the next cycle from the current ||r||.
template <int DIM, bool FUSED>
__global__ void __launch_bounds__(NT) k_spmv_pq(Ctx c, const double *__restrict__ s,
                                                const double *__restrict__ pold,
                                                double *__restrict__ pnew, int cons) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const NodeBlk nbk = node_block(c);
  const int b = nbk.b, blk = nbk.blk;
  InstState *st = c.st + b;
  // finished or pending instances are skipped at the first store (see k_sweep)
  if (c.batch > 1 && (st->done | st->pending)) return;
  const int skip = st->done | st->pending;
  double beta = st->beta;
  if (FUSED && cons && c.cons) {
    if (skip) return;
    const double trs = consume_partials(slot(c, b, SLOT_RHO), c.nbn, lds);
    if (!(trs > 0.0)) {
      if (blk == 0 && threadIdx.x == 0) breakdown(st, trs);
      return;
    }
    beta = beta_of(st, trs);
  }
  const int node = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  const double *sb = s + off, *pb = pold + off;
  double *pn = pnew + off;
  // the direction p = s + beta p_old (or the p formed by k_pdir) around the
  // block, in LDS when staged
  extern __shared__ double xlds_dyn[];
  double *xs = (double *)xlds_dyn;
  long long xlo = 0;
  if (c.xwin) {
    if (FUSED) xlo = stage_x<DIM, double>(c, blk, xs, [sb, pb, beta](size_t i) { return pdir(sb[i], pb, i, beta); });
    else xlo = stage_x<DIM, double>(c, blk, xs, [pn](size_t i) { return pn[i]; });
  }
  double pq = 0.0;
  const size_t r0 = (size_t)node * DIM;
  double kp[DIM], pv[DIM];
  if (node < c.nn) {
    const double *vals = c.vals + (size_t)b * c.vstride;
    if (c.xwin) {
      node_dot<DIM>(c.colblk, vals, [xs, xlo](size_t i) { return xs[i - xlo]; }, node, c.n, c.nn, kp);
#pragma unroll
      for (int r = 0; r < DIM; ++r) pv[r] = xs[r0 + r - xlo];
    } else if (FUSED) {
      const auto pdir_at = [sb, pb, beta](size_t i) { return pdir(sb[i], pb, i, beta); };
      node_dot<DIM, double, decltype(pdir_at), DIM == 3 ? 3 : 9>(c.colblk, vals, pdir_at, node, c.n, c.nn, kp);
#pragma unroll
      for (int r = 0; r < DIM; ++r) pv[r] = pdir(sb[r0 + r], pb, r0 + r, beta);
    } else {
      node_dot<DIM>(c.colblk, vals, [pn](size_t i) { return pn[i]; }, node, c.n, c.nn, kp);
#pragma unroll
      for (int r = 0; r < DIM; ++r) pv[r] = pn[r0 + r];
    }
  }
  if (skip) return;
  if (blk == 0 && threadIdx.x == 0) st->scale = cycle_scale(c, st->rr);
  if (node < c.nn) {
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
      if (FUSED) pn[r0 + r] = pv[r];
      c.q[off + r0 + r] = kp[r];
      pq += pv[r] * kp[r];
    }
  }
  double dummy = 0.0;
  block_sum2(pq, dummy, lds);
  if (threadIdx.x == 0) put_partial(slot(c, b, SLOT_GAMMA) + blk, pq);
  if (c.cons || !arrive_last(site(c, b, CNT_D), blk, c.nbn, &flag)) return;
  // producer side (large grids): alpha here
  const double g = reduce_partials(slot(c, b, SLOT_GAMMA), c.nbn, 1, lds);
  if (threadIdx.x == 0) {
    st->gamma = g;
    if (!(g > 0.0)) breakdown(st, g);
    st->alpha = st->rho / g;
  }
}

// p = s + beta p_old (the unfused form of the direction update); beta as in
// k_spmv_pq.
__global__ void __launch_bounds__(NT) k_pdir(Ctx c, const double *__restrict__ s,
                                             const double *__restrict__ pold,
                                             double *__restrict__ pnew, int cons) {
  __shared__ double lds[NWAVE];
  const int b = inst_id();
  InstState *st = c.st + b;
  if (st->done || st->pending) return;
  double beta = st->beta;
  if (cons && c.cons) {
    const double trs = consume_partials(slot(c, b, SLOT_RHO), c.nbn, lds);
    if (!(trs > 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) breakdown(st, trs);
      return;
    }
    beta = beta_of(st, trs);
  }
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= c.n) return;
  const size_t off = (size_t)b * c.n;
  pnew[off + row] = pdir(s[off + row], pold + off, row, beta);
}

// alpha = rho / p^T q from the partials of the outer SpMV (and, with a
// preconditioner, rho = r^T s from the cycle's), then u += alpha p,
// r -= alpha q, ||r||^2 (and r^T s_old for the flexible beta); with a
// preconditioner also the next cycle's input and, for mode 1, its first
// pre-relaxation sweep.  Last block: convergence, iteration limit,
// non-finite checks, and the state the next direction update reads (rho,
// the restart flag cleared); without a preconditioner (mode 0) s = r, so
// rho and beta are formed here.  A pending instance (served
// solve whose true residual f - K u sits in q) takes r = q instead, leaves
// u and the iteration count alone, and restarts from there: this is the
// first step of a newly admitted solve and of a residual replacement.
template <typename T>
__global__ void __launch_bounds__(NT) k_update(Ctx c, int mode, const double *__restrict__ p) {
  const int have_prec = mode != 0;
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const int b = inst_id();
  InstState *st = c.st + b;
  if (c.batch > 1 && st->done) return;
  const int done = st->done;   // one instance: checked at the first store (see k_sweep)
  const bool pend = st->pending != 0;
  const int blk = blockIdx.x;
  const int row = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  const bool pr = have_prec && st->beta_kind == POD2G_BETA_PR && !pend;
  double rr = 0.0, rs = 0.0;
  double uv = 0.0, pv = 0.0, rv0 = 0.0, qv = 0.0;
  if (row < c.n) {
    uv = c.u[off + row];
    pv = p[off + row];
    rv0 = c.r[off + row];
    qv = c.q[off + row];
  }
  if (done) return;
  double alpha = st->alpha, g = 0.0, rho = 0.0;
  if (!pend && c.cons) {
    g = consume_partials(slot(c, b, SLOT_GAMMA), c.nbn, lds);
    rho = have_prec ? consume_partials(slot(c, b, SLOT_RHO), c.nbn, lds) : st->rho;
    if (!(g > 0.0)) {
      if (blk == 0 && threadIdx.x == 0) { st->gamma = g; breakdown(st, g); }
      return;
    }
    alpha = rho / g;
  }
  if (row < c.n) {
    double rv;
    if (pend) {
      rv = qv;
    } else {
      c.u[off + row] = uv + alpha * pv;
      rv = rv0 - alpha * qv;
    }
    c.r[off + row] = rv;
    rr = rv * rv;
    if (pr) rs = rv * c.s[off + row];
    if (have_prec) {
      const T bv = (T)(rv * st->scale);
      if (sizeof(T) == 4) ((float *)c.b32)[off + row] = (float)bv;
      if (mode == 1) ((T *)c.xa)[off + row] = (T)c.omega * ((const T *)c.sdinv)[off + row] * bv;
    }
  }
  block_sum2(rr, rs, lds);
  if (threadIdx.x == 0) { put_partial(slot(c, b, 0) + blk, rr); put_partial(slot(c, b, 1) + blk, rs); }
  if (!arrive_last(site(c, b, CNT_E), blk, c.nb, &flag)) return;
  const double trr = reduce_partials(slot(c, b, 0), c.nb, 1, lds);
  const double trs = pr ? reduce_partials(slot(c, b, 1), c.nb, 1, lds) : 0.0;
  if (threadIdx.x == 0) {
    if (pend) {
      st->pending = 0;
    } else {
      st->iter += 1;
      if (c.cons) {
        st->gamma = g;
        st->alpha = alpha;
        if (have_prec) {
          st->rho = rho;
          st->restart = 0;
        }
      }
    }
    st->rr = trr;
    st->rs_prev = trs;
    if (!finite(trr)) { st->done = 1; st->status = POD2G_ENAN; }
    else if (trr <= st->tol2) { st->done = 1; st->status = POD2G_OK; }
    else if (st->iter >= st->maxit) { st->done = 1; st->status = POD2G_EMAXIT; }
    if (!have_prec) {
      st->beta = pend ? 0.0 : trr / st->rho;
      st->rho = trr;
    }
  }
}

// k_update (mode 1) fused with the second pre-relaxation sweep, one thread
// per node.  The first sweep starts from x = 0 and is pointwise,
// x1 = omega D^-1 b with b = scale (r - alpha q) (b = scale q for a pending
// instance), so the second sweep x2 = x1 + omega D^-1 (b - K x1) forms x1
// at the neighbours from r, q and D^-1 there, with the expressions of the
// owned rows, instead of reading a stored x1.  The neighbours' r must be
// the old one, so the new residual goes to the other buffer (rin and rout
// swap roles every iteration).  Writes u, rout, (FP32 b) and x2 to xout;
// the ||r||^2 (and r^T s_old) reduction and its last workgroup are those
// of k_update, over node blocks.
template <int DIM, typename T>
__global__ void __launch_bounds__(NT) k_update_sweep(Ctx c, const double *__restrict__ p,
                                                     const double *__restrict__ rin,
                                                     double *__restrict__ rout, T *__restrict__ xout) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const NodeBlk nbk = node_block(c);
  const int b = nbk.b, blk = nbk.blk;
  InstState *st = c.st + b;
  if (c.batch > 1 && st->done) return;
  const int done = st->done;   // one instance: checked at the first store (see k_sweep)
  const bool pend = st->pending != 0;
  const bool pr = st->beta_kind == POD2G_BETA_PR && !pend;
  const int node = blk * NT + threadIdx.x;
  const bool own = node < c.nn;
  const size_t off = (size_t)b * c.n;
  const size_t r0 = off + (size_t)node * DIM;
  double uv[DIM], pv[DIM], rv0[DIM], qv[DIM];
#pragma unroll
  for (int r = 0; r < DIM; ++r) {
    uv[r] = own ? c.u[r0 + r] : 0.0;
    pv[r] = own ? p[r0 + r] : 0.0;
    rv0[r] = own ? rin[r0 + r] : 0.0;
    qv[r] = own ? c.q[r0 + r] : 0.0;
  }
  if (done) return;
  double alpha = st->alpha, g = 0.0, rho = 0.0;
  if (!pend && c.cons) {
    g = consume_partials(slot(c, b, SLOT_GAMMA), c.nbn, lds);
    rho = consume_partials(slot(c, b, SLOT_RHO), c.nbn, lds);
    if (!(g > 0.0)) {
      if (blk == 0 && threadIdx.x == 0) { st->gamma = g; breakdown(st, g); }
      return;
    }
    alpha = rho / g;
  }
  const double scale = st->scale;
  const T om = (T)c.omega;
  const double *rb = rin + off, *qb = c.q + off;
  const T *db = (const T *)c.sdinv + off;
  double rr = 0.0, rs = 0.0;
  if (own) {
    T kx[DIM];
    const T *vals = (const T *)c.svals + (size_t)b * c.vstride;
    // x1 at any row i, from r, q and D^-1 there
    const auto x1_at = [=](size_t i) {
      const double rvi = pend ? qb[i] : rb[i] - alpha * qb[i];
      return om * db[i] * (T)(rvi * scale);
    };
    node_dot<DIM, T, decltype(x1_at), DIM == 3 ? 3 : 9>(c.colblk, vals, x1_at, node, c.n, c.nn, kx);
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
      const size_t row = r0 + r;
      double rv;
      if (pend) {
        rv = qv[r];
      } else {
        c.u[row] = uv[r] + alpha * pv[r];
        rv = rv0[r] - alpha * qv[r];
      }
      rout[row] = rv;
      rr += rv * rv;
      if (pr) rs += rv * c.s[row];
      const T bv = (T)(rv * scale);
      if (sizeof(T) == 4) ((float *)c.b32)[row] = (float)bv;
      const T dv = ((const T *)c.sdinv)[row];
      const T rhs = sizeof(T) == 8 ? (T)rv : bv;   // the cycle's right-hand side (see cycle_rhs)
      const T x1 = om * dv * bv;
      xout[row] = fma_t(om * dv, rhs - kx[r], x1);   // as in k_sweep, bit for bit
    }
  }
  block_sum2(rr, rs, lds);
  if (threadIdx.x == 0) { put_partial(slot(c, b, 0) + blk, rr); put_partial(slot(c, b, 1) + blk, rs); }
  if (!arrive_last(site(c, b, CNT_E), blk, c.nbn, &flag)) return;
  const double trr = reduce_partials(slot(c, b, 0), c.nbn, 1, lds);
  const double trs = pr ? reduce_partials(slot(c, b, 1), c.nbn, 1, lds) : 0.0;
  if (threadIdx.x == 0) {
    if (pend) {
      st->pending = 0;
    } else {
      st->iter += 1;
      if (c.cons) {
        st->gamma = g;
        st->alpha = alpha;
        st->rho = rho;
        st->restart = 0;
      }
    }
    st->rr = trr;
    st->rs_prev = trs;
    if (!finite(trr)) { st->done = 1; st->status = POD2G_ENAN; }
    else if (trr <= st->tol2) { st->done = 1; st->status = POD2G_OK; }
    else if (st->iter >= st->maxit) { st->done = 1; st->status = POD2G_EMAXIT; }
  }
}

// ---------------------------------------------------------------------------
// Batched products with the shared basis (mixed cycle, FP32 on MFMA).
// v_mfma_f32_16x16x4f32 operand layout (one 64-lane wave): A[i][kk] in lane
// i + 16 kk, B[kk][j] in lane j + 16 kk, D[i][j] in lane j + 16 (i / 4),
// register i % 4.
// ---------------------------------------------------------------------------

// Restriction for all instances at once: C[j][b] = sum_rows P[j][row] R[b][row]
// with R the residuals r'_b (FP32, [batch][n]), on MFMA with the operands
// loaded straight from memory.  In step s of a group of four MFMA steps over
// rows r0 .. r0 + 15, lane i + 16 kk holds A[i][kk] = P[j0 + i][r0 + 4 kk + s]
// and B[kk][i] = R[b0 + i][r0 + 4 kk + s]: a lane's operands of the four
// steps are four consecutive floats of one row of P (or R), one 16-byte
// load, and the contraction over the group's 16 rows is complete.  No LDS
// staging and no barriers in the loop: every wave accumulates all output
// tiles over its own contiguous share of the row groups, with GRP groups'
// loads in flight together.  Output rows j >= k and columns b >= batch (and
// finished instances) are computed from clamped addresses and never used;
// rows >= n are zeroed.  The workgroup's four waves are summed in FP64 into
// one partial per output (k_ptr_sum sums the workgroups, k_coarse_b applies
// the coarse solves).  VEC: n % 4 == 0, so a group's 16-byte loads are
// aligned and lie wholly below or wholly above n.
constexpr int PTR_GRP = 2;        // 16-row groups per wave iteration (default; tunable)

template <bool VEC>
__device__ __forceinline__ f4 ptr_load(const float *__restrict__ row_base, int r, int n) {
  if (VEC) {
    const bool ok = r < n;
    f4 v = *(const f4 *)(row_base + (ok ? r : 0));
    return ok ? v : f4{0.f, 0.f, 0.f, 0.f};
  } else {
    f4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool ok = r + e < n;
      const float x = row_base[ok ? r + e : 0];
      v[e] = ok ? x : 0.f;
    }
    return v;
  }
}

// TJ = ceil(k / 16) basis tiles, TB = ceil(batch / 16) batch tiles, GRP
// row groups loaded together (a schedule choice: each wave still adds its
// groups in order, so every GRP gives the same bits).
template <int TJ, int TB, bool VEC, int GRP>
__global__ void __launch_bounds__(NT) k_ptr_b(Ctx c, const float *__restrict__ R) {
  __shared__ float Cs[NWAVE][TJ * 16][TB * 16];   // the waves' tiles (at most 32 KB)
  __shared__ int nlive;
  const int B = c.batch, k = c.k, n = c.n;
  const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  if (threadIdx.x == 0) nlive = 0;
  __syncthreads();
  if (threadIdx.x < B && !c.st[threadIdx.x].done) atomicAdd(&nlive, 1);
  __syncthreads();
  if (nlive == 0) return;
  f4 acc[TJ][TB];
#pragma unroll
  for (int t = 0; t < TJ; ++t)
#pragma unroll
    for (int u = 0; u < TB; ++u) acc[t][u] = f4{0.f, 0.f, 0.f, 0.f};
  const int li = lane & 15, kk = lane >> 4;
  // operand rows of this lane: basis row j (clamped to k - 1) per j tile,
  // residual row b (clamped to batch - 1) per batch tile
  const float *P = (const float *)c.sP;
  const float *pa[TJ];
  const float *rb[TB];
#pragma unroll
  for (int t = 0; t < TJ; ++t) pa[t] = P + (size_t)min(t * 16 + li, k - 1) * n;
#pragma unroll
  for (int u = 0; u < TB; ++u) rb[u] = R + (size_t)min(u * 16 + li, B - 1) * n;
  // this wave's share of the 16-row groups
  const int g = xcd_block(blockIdx.x, c.bgrid);
  const long long ngroups = (n + 15) / 16, nwaves = (long long)c.bgrid * NWAVE;
  const long long per = (ngroups + nwaves - 1) / nwaves;
  const long long wv = (long long)g * NWAVE + w;
  const long long gbeg = wv * per, gend = min(ngroups, gbeg + per);
  for (long long g0 = gbeg; g0 < gend; g0 += GRP) {
    f4 a[GRP][TJ], bv[GRP][TB];
#pragma unroll
    for (int q = 0; q < GRP; ++q) {
      // a group past the share (its rows may exist) or past n loads zeros
      const int r = (g0 + q < gend) ? (int)((g0 + q) * 16) + 4 * kk : n;
#pragma unroll
      for (int t = 0; t < TJ; ++t) a[q][t] = ptr_load<VEC>(pa[t], r, n);
#pragma unroll
      for (int u = 0; u < TB; ++u) bv[q][u] = ptr_load<VEC>(rb[u], r, n);
    }
#pragma unroll
    for (int q = 0; q < GRP; ++q)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int t = 0; t < TJ; ++t)
#pragma unroll
          for (int u = 0; u < TB; ++u)
            acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q][t][s4], bv[q][u][s4], acc[t][u], 0, 0, 0);
  }
  // D[i][jb] of tile (t, u) sits in lane jb + 16 (i / 4), register i % 4
#pragma unroll
  for (int t = 0; t < TJ; ++t)
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cs[w][t * 16 + 4 * kk + v][u * 16 + li] = acc[t][u][v];
  __syncthreads();
  double *gp = c.bpart + (size_t)g * k * B;
  for (int o = threadIdx.x; o < k * B; o += NT) {
    const int j = o / B, b = o % B;
    double sum = 0.0;
#pragma unroll
    for (int ww = 0; ww < NWAVE; ++ww) sum += (double)Cs[ww][j][b];
    gp[o] = sum;
  }
}

// r_c of every (j, b): the workgroup partials of k_ptr_b summed by 16 threads
// per output (strided shares, then a fixed 16-lane tree).
constexpr int PTR_TPO = 16;   // threads per output

__global__ void __launch_bounds__(NT) k_ptr_sum(Ctx c) {
  const int B = c.batch, k = c.k;
  const int o = (blockIdx.x * NT + threadIdx.x) / PTR_TPO, q = threadIdx.x % PTR_TPO;
  double v = 0.0;
  if (o < k * B) v = strided_sum_wide(c.bpart + o, q, c.bgrid, PTR_TPO, k * B);
#pragma unroll
  for (int d = PTR_TPO / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, PTR_TPO);
  double *rc = c.bpart + (size_t)c.bgrid * k * B;   // k * B sums after the partials
  if (q == 0 && o < k * B) rc[o] = v;
}

// Coarse solves of the batched restriction, one workgroup per live
// instance: its factor and its r_c in LDS, then e_c = Linv^T (Linv r_c).
__global__ void __launch_bounds__(NT) k_coarse_b(Ctx c) {
  __shared__ double Ls[MAXK * MAXK];
  __shared__ double r[MAXK], y[MAXK];
  const int b = blockIdx.x, B = c.batch, k = c.k, t = threadIdx.x;
  if (c.st[b].done) return;
  const double *Li = c.Linv + (size_t)b * k * k;
  const double *rc = c.bpart + (size_t)c.bgrid * k * B;
  for (int i = t; i < k * k; i += NT) Ls[i] = Li[i];
  if (t < k) r[t] = rc[(size_t)t * B + b];
  __syncthreads();
  if (t < k) {
    double v = 0.0;
    for (int j = 0; j <= t; ++j) v += Ls[t * k + j] * r[j];
    y[t] = v;
  }
  __syncthreads();
  if (t < k) {
    double e = 0.0;
    for (int j = t; j < k; ++j) e += Ls[j * k + t] * y[j];
    c.ec[(size_t)b * MAXK + t] = e;
  }
}

// Prolongation and correction for all instances of a 256-row block:
// X_out[b][row] = X_in[b][row] + sum_j P[j][row] E[j][b] with the k x B
// product on MFMA (FP32), staged through LDS so the writes are coalesced.
// With rp (the restricted residual r', [batch][n]) the kernel also applies
// the first post-relaxation sweep: since b - K (x + P e_c) = r' - (K P) e_c,
// x_out = x + P e_c + omega D^-1 (r' - (K P) e_c) reads the instance's K P
// (k values per row) instead of its K and the gathered x.
__global__ void __launch_bounds__(NT) k_prolong_b(Ctx c, const float *__restrict__ xin,
                                                  float *__restrict__ xout,
                                                  const float *__restrict__ rp) {
  __shared__ float E[MAXK][MAXB];           // 8 KB
  __shared__ float Out[MAXB][NT];           // 32 KB
  __shared__ int live[MAXB];
  __shared__ int nlive;
  const int B = c.batch, k = c.k, n = c.n;
  const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  if (threadIdx.x < B) live[threadIdx.x] = !c.st[threadIdx.x].done;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = 0;
    for (int b = 0; b < B; ++b) m += live[b];
    nlive = m;
  }
  {
    // coarse corrections into LDS: all loads first (addresses clamped into
    // range, so none is guarded), then the stores with the padding zeroed
    constexpr int EU = MAXK * MAXB / NT;
    float ev[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int t = threadIdx.x + u * NT;
      const int j = t / MAXB, b = t % MAXB;
      ev[u] = (float)c.ec[(size_t)(b < B ? b : B - 1) * MAXK + (j < k ? j : k - 1)];
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int t = threadIdx.x + u * NT;
      const int j = t / MAXB, b = t % MAXB;
      E[j][b] = (j < k && b < B) ? ev[u] : 0.f;
    }
  }
  __syncthreads();
  if (nlive == 0) return;
  const int blk = xcd_block(blockIdx.x, c.nb);
  const int rw0 = blk * NT + w * WAVE;
  const float *P = (const float *)c.sP;
  const int tb = (B + 15) / 16, ks = (k + 3) / 4;
  for (int tr = 0; tr < WAVE / 16; ++tr) {
    // this row tile's basis entries for all k, loads in flight together
    const int row_a = rw0 + 16 * tr + (lane & 15);
    float av[MAXK / 4];
#pragma unroll
    for (int s4 = 0; s4 < MAXK / 4; ++s4) {
      const int kk = 4 * s4 + (lane >> 4);
      av[s4] = (s4 < ks && kk < k && row_a < n) ? P[(size_t)kk * n + row_a] : 0.f;
    }
    for (int t2 = 0; t2 < tb; ++t2) {
      f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s4 = 0; s4 < MAXK / 4; ++s4) {
        if (s4 < ks) {
          const int kk = 4 * s4 + (lane >> 4);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s4], E[kk][t2 * 16 + (lane & 15)], acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int bb = t2 * 16 + (lane & 15);
        if (bb < MAXB) Out[bb][w * WAVE + 16 * tr + 4 * (lane >> 4) + v] = acc[v];
      }
    }
  }
  __syncthreads();
  const int row = blk * NT + threadIdx.x;
  if (row >= n) return;
  const float *dinv = (const float *)c.sdinv;
  // two instances at a time, so that both instances' loads are in flight
  // together (each instance's arithmetic does not depend on its partner)
  for (int b0 = 0; b0 < B; b0 += 2) {
    const int b1 = b0 + 1;   // < MAXB: E and Out hold zeros past the batch
    // the same for the whole workgroup: scalar branches, so that the loads
    // inside are not guarded one by one
    const bool l0 = __builtin_amdgcn_readfirstlane(live[b0]) != 0;
    const bool l1 = b1 < B && __builtin_amdgcn_readfirstlane(live[b1]) != 0;
    if (!l0 && !l1) continue;
    const size_t o0 = (size_t)b0 * n, o1 = (size_t)b1 * n;
    float xv0 = 0.f, xv1 = 0.f, d0 = 0.f, d1 = 0.f, dv0 = 0.f, dv1 = 0.f;
    if (l0) {
      xv0 = xin ? xin[o0 + row] : 0.f;
      if (rp) { d0 = rp[o0 + row]; dv0 = dinv[o0 + row]; }
    }
    if (l1) {
      xv1 = xin ? xin[o1 + row] : 0.f;
      if (rp) { d1 = rp[o1 + row]; dv1 = dinv[o1 + row]; }
    }
    xv0 += Out[b0][threadIdx.x];
    xv1 += Out[b1][threadIdx.x];
    if (rp) {
      // up to 32 loads of K P per instance in flight before their products
      // (one round for k <= 32)
      constexpr int KC = 32;
      const float *kp0 = c.KP32 + (size_t)b0 * k * n + row;
      const float *kp1 = c.KP32 + (size_t)(l1 ? b1 : b0) * k * n + row;
      for (int j0 = 0; j0 < k; j0 += KC) {
        // K P rows past k are read at k - 1 (in range) and meet zeros in E
        float kv0[KC], kv1[KC];
        if (l0) {
#pragma unroll
          for (int u = 0; u < KC; ++u) kv0[u] = kp0[(size_t)(j0 + u < k ? j0 + u : k - 1) * n];
        } else {
#pragma unroll
          for (int u = 0; u < KC; ++u) kv0[u] = 0.f;
        }
        if (l1) {
#pragma unroll
          for (int u = 0; u < KC; ++u) kv1[u] = kp1[(size_t)(j0 + u < k ? j0 + u : k - 1) * n];
        } else {
#pragma unroll
          for (int u = 0; u < KC; ++u) kv1[u] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < KC; ++u) {
          const int j = j0 + u < MAXK ? j0 + u : 0;
          d0 -= kv0[u] * E[j][b0];
          d1 -= kv1[u] * E[j][b1];
        }
      }
      xv0 += (float)c.omega * dv0 * d0;
      xv1 += (float)c.omega * dv1 * d1;
    }
    if (l0) xout[o0 + row] = xv0;
    if (l1) xout[o1 + row] = xv1;
  }
}

// Outcome of a served solve whose true residual rr_true = ||f - K u||^2 was
// just formed (thread 0 of the last block).  A newly admitted instance
// learns ||f|| and either stops at x0 or starts; a stopped one either
// finishes (result published in info) or, if the recursive residual met the
// tolerance but the true one does not, restarts from the true residual, as
// the exit check of the one-shot solve does.
__device__ void serve_decide(const Ctx &c, InstState *st, int b, double t, double tf, bool fresh) {
  bool restart;
  if (fresh) {
    st->fresh = 0;
    st->ff = tf;
    st->tol2 *= tf;   // held rtol^2 since admission
    if (!finite(t) || !finite(tf)) { st->status = POD2G_ENAN; restart = false; }
    else { st->status = POD2G_OK; restart = t > st->tol2; }
  } else {
    if (!finite(t)) st->status = POD2G_ENAN;
    restart = st->status == POD2G_OK && st->iter < st->maxit && t > st->tol2 && st->iter > 0;
    if (!restart && st->status == POD2G_OK && t > st->tol2) st->status = POD2G_EMAXIT;
  }
  if (restart) {
    st->pending = 1;
    st->done = 0;
    st->restart = 1;
    st->beta = 0.0;
    st->rr = t;
    st->scale = cycle_scale(c, t);
    return;
  }
  st->done = 1;
  st->checked = 1;
  pod2g_slot_info in;
  in.done = 1;
  in.iter = st->iter;
  in.status = st->status;
  in.pad = 0;
  in.relres = st->ff > 0.0 ? sqrt(t / st->ff) : 0.0;
  c.info[b] = in;
}

// q = f - K u with ||q||^2.  gate == 0: every instance, done or not (exit
// check of the one-shot solve).  gate == 1 (served solves): only instances
// that stopped and are not checked yet, which includes the newly admitted
// ones (they also reduce ||f||^2); the last block decides their outcome.
template <int DIM>
__global__ void __launch_bounds__(NT) k_true_resid(Ctx c, int gate) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const int b = inst_id();
  InstState *st = c.st + b;
  if (gate && !(st->done && !st->checked)) return;
  const bool fresh = gate && st->fresh;
  const int blk = xcd_block(blockIdx.x, c.nb);
  const int row = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  double rr = 0.0, ff = 0.0;
  if (row < c.n) {
    const double kx = row_dot<DIM>(c.colblk, c.vals + (size_t)b * c.vstride, c.u + off, row,
                                   row / DIM, c.n, c.nn);
    const double fv = c.f[row];
    const double rv = fv - kx;
    c.q[off + row] = rv;
    rr = rv * rv;
    ff = fv * fv;
  }
  block_sum2(rr, ff, lds);
  if (threadIdx.x == 0) {
    put_partial(slot(c, b, 0) + blk, rr);
    if (fresh) put_partial(slot(c, b, 1) + blk, ff);
  }
  if (!arrive_last(site(c, b, CNT_A), blk, c.nb, &flag)) return;
  const double t = reduce_partials(slot(c, b, 0), c.nb, 1, lds);
  const double tf = fresh ? reduce_partials(slot(c, b, 1), c.nb, 1, lds) : 0.0;
  if (threadIdx.x == 0) {
    st->rr_true = t;
    if (gate) serve_decide(c, st, b, t, tf, fresh);
  }
}

// Standalone two-grid solver (the POD-2G scheme of Sec. 3.3 iterated on its
// own, as in the Sec. 4 comparisons): u += s after the cycle s = B r ...
__global__ void __launch_bounds__(NT) k_stat_update(Ctx c) {
  const int b = inst_id();
  if (c.st[b].done) return;
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= c.n) return;
  const size_t off = (size_t)b * c.n;
  c.u[off + row] += c.s[off + row];
}

// ... then r = f - K u (one thread per node) with ||r||^2; the last block
// counts the iteration, tests ||r|| <= rtol ||f|| and the iteration limit,
// and sets the next cycle's input scale.
template <int DIM>
__global__ void __launch_bounds__(NT) k_stat_resid(Ctx c) {
  __shared__ double lds[2 * NWAVE];
  __shared__ int flag;
  const NodeBlk nbk = node_block(c);
  const int b = nbk.b, blk = nbk.blk;
  InstState *st = c.st + b;
  if (st->done) return;
  const int node = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  const double *ub = c.u + off;
  extern __shared__ double xlds_dyn[];
  double *xs = (double *)xlds_dyn;
  const long long xlo = c.xwin ? stage_x<DIM, double>(c, blk, xs, [ub](size_t i) { return ub[i]; }) : 0;
  double rr = 0.0;
  if (node < c.nn) {
    double kx[DIM];
    if (c.xwin)
      node_dot<DIM>(c.colblk, c.vals + (size_t)b * c.vstride,
                    [xs, xlo](size_t i) { return xs[i - xlo]; }, node, c.n, c.nn, kx);
    else
      node_dot<DIM>(c.colblk, c.vals + (size_t)b * c.vstride, [ub](size_t i) { return ub[i]; },
                    node, c.n, c.nn, kx);
    const size_t r0 = (size_t)node * DIM;
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
      const double rv = c.f[r0 + r] - kx[r];
      c.r[off + r0 + r] = rv;
      rr += rv * rv;
    }
  }
  double dummy = 0.0;
  block_sum2(rr, dummy, lds);
  if (threadIdx.x == 0) put_partial(slot(c, b, 0) + blk, rr);
  if (!arrive_last(site(c, b, CNT_A), blk, c.nbn, &flag)) return;
  const double trr = reduce_partials(slot(c, b, 0), c.nbn, 1, lds);
  if (threadIdx.x == 0) {
    st->iter += 1;
    st->rr = trr;
    st->rr_true = trr;
    st->scale = cycle_scale(c, trr);
    if (!finite(trr)) { st->done = 1; st->status = POD2G_ENAN; }
    else if (trr <= st->tol2) { st->done = 1; st->status = POD2G_OK; }
    else if (st->iter >= st->maxit) { st->done = 1; st->status = POD2G_EMAXIT; }
  }
}

// Residual replacement for the instances flagged by the host: r = q,
// CG restarts (beta = 0) and the instance becomes live again.
__global__ void __launch_bounds__(NT) k_replace(Ctx c, const int *__restrict__ flags, int have_prec) {
  const int b = inst_id();
  if (!flags[b]) return;
  const int row = blockIdx.x * NT + threadIdx.x;
  const size_t off = (size_t)b * c.n;
  if (row < c.n) c.r[off + row] = c.q[off + row];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    InstState *st = c.st + b;
    st->rr = st->rr_true;
    st->scale = cycle_scale(c, st->rr_true);
    st->done = 0;
    st->restart = 1;
    st->beta = 0.0;
    if (!have_prec) st->rho = st->rr_true;
  }
}

// ---------------------------------------------------------------------------
// Gauss-Seidel relaxation in multicolour node order (the relaxation of
// Alg. 2 in the Gauss-Seidel form the paper analyses).  Node (i, j[, l]) has
// colour (i mod 2) + 2 (j mod 2) [+ 4 (l mod 2)]; nodes of one colour share
// no matrix entry, so one launch updates a colour, one thread per node,
// its DIM unknowns in turn (reversed in backward sweeps) against the
// current values of its own unknowns and its neighbours'.
// ---------------------------------------------------------------------------
struct Colour {
  int i0, ni, j0, nj, l0, nl;   // first index and count per grid direction
};

// Free nodes: 2D i in [1, N] (x = 0 clamped), j in [0, N];
// 3D i, j in [0, N], l in [1, N] (z = 0 clamped).
static Colour colour_of(int dim, int N, int col) {
  const int px = col & 1, py = (col >> 1) & 1, pz = (col >> 2) & 1;
  auto span = [N](int lo) { return lo <= N ? (N - lo) / 2 + 1 : 0; };
  Colour c;
  if (dim == 2) {
    c.i0 = px ? 1 : 2; c.ni = span(c.i0);
    c.j0 = py;         c.nj = span(c.j0);
    c.l0 = 0;          c.nl = 1;
  } else {
    c.i0 = px;         c.ni = span(c.i0);
    c.j0 = py;         c.nj = span(c.j0);
    c.l0 = pz ? 1 : 2; c.nl = span(c.l0);
  }
  return c;
}

template <int DIM, typename T, bool BACK>
__global__ void __launch_bounds__(NT) k_gs_colour(Ctx c, const T *__restrict__ rhs_in,
                                                  T *__restrict__ x, Colour col) {
  constexpr int S = Stencil<DIM>::S, SC = S / 2;   // SC: the node's own block
  const int b = blockIdx.y;
  if (c.st && c.st[b].done) return;
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= col.ni * col.nj * col.nl) return;
  const int i = col.i0 + 2 * (t % col.ni);
  const int rest = t / col.ni;
  const int j = col.j0 + 2 * (rest % col.nj);
  const int node = DIM == 2 ? j * c.N + (i - 1)
                            : ((col.l0 + 2 * (rest / col.nj)) - 1) * (c.N + 1) * (c.N + 1) +
                                  j * (c.N + 1) + i;
  const size_t off = (size_t)b * c.n;
  const T *vb = (const T *)c.svals + (size_t)b * c.vstride;
  const size_t ns = (size_t)c.n + DIM;
  T *xb = x + off;
  T acc[DIM];
#pragma unroll
  for (int r = 0; r < DIM; ++r) acc[r] = T(0);
  // the other slots in order (lower, then upper past the own block)
#pragma unroll
  for (int s = 0; s < SC; ++s) node_slot<DIM, T, true>(c.colblk, vb, [xb](size_t i) { return xb[i]; },
                                                       s, node, c.nn, ns, acc);
#pragma unroll
  for (int s = SC + 1; s < S; ++s) node_slot<DIM, T, false>(c.colblk, vb, [xb](size_t i) { return xb[i]; },
                                                            s, node, c.nn, ns, acc);
  T xo[DIM], kc[DIM][DIM];
#pragma unroll
  for (int r = 0; r < DIM; ++r) xo[r] = xb[(size_t)node * DIM + r];
  load_block<DIM, T, false>(vb, SC, node, node, c.nn, ns, kc);
  const T *rhs = (rhs_in ? rhs_in + off : cycle_rhs<T>(c, off)) + (size_t)node * DIM;
  const T *dv = (const T *)c.sdinv + off + (size_t)node * DIM;
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    const int r = BACK ? DIM - 1 - q : q;
    T a = acc[r];
#pragma unroll
    for (int bc = 0; bc < DIM; ++bc) a += kc[r][bc] * xo[bc];
    xo[r] += dv[r] * (rhs[r] - a);
  }
#pragma unroll
  for (int r = 0; r < DIM; ++r) xb[(size_t)node * DIM + r] = xo[r];
}

template <typename T>
__global__ void __launch_bounds__(NT) k_zero(T *__restrict__ x, size_t count) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT)
    x[i] = T(0);
}

// Served solves: a free slot is stopped and checked, so no kernel touches
// it; an admitted one is stopped, unchecked and fresh, so the next gated
// true-residual pass forms r0 = f - K x0 and ||f|| and starts it.
__global__ void k_serve_free(InstState *st, Arrival *arr, pod2g_slot_info *info, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  zero_arrivals(arr + (size_t)b * NSITE, NSITE, 0, 1);
  InstState s;
  memset(&s, 0, sizeof(s));
  s.done = 1;
  s.checked = 1;
  s.scale = 1.0;
  st[b] = s;
  pod2g_slot_info in;
  memset(&in, 0, sizeof(in));
  in.done = 1;
  info[b] = in;
}

__global__ void k_serve_admit(InstState *st, Arrival *arr, pod2g_slot_info *info, int b, double rtol,
                              int maxit, int beta_kind, const int *setup_status) {
  zero_arrivals(arr + (size_t)b * NSITE, NSITE, threadIdx.x, blockDim.x);
  if (threadIdx.x != 0) return;
  InstState s;
  memset(&s, 0, sizeof(s));
  s.maxit = maxit;
  s.beta_kind = beta_kind;
  s.restart = 1;
  s.scale = 1.0;
  s.tol2 = rtol * rtol;
  s.done = 1;
  pod2g_slot_info in;
  memset(&in, 0, sizeof(in));
  const int ss = setup_status ? setup_status[b] : 0;
  if (ss != 0) {
    s.checked = 1;
    s.status = ss;
    in.done = 1;
    in.status = ss;
  } else {
    s.fresh = 1;
  }
  st[b] = s;
  info[b] = in;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Per-call timing: the first per_call launches of the timer's kernel in a
// solve go through hipExtLaunchKernel, whose start/stop events receive the
// dispatch's own begin/end timestamps (the clock a kernel trace reads).
struct Tm {
  pod2g_timer *t;
  int used;
};

template <typename F, typename... Args>
static void launch(Tm *tm, int id, F kernel, dim3 grid, dim3 block, unsigned shm,
                   hipStream_t s, Args... args) {
  if (tm && tm->t && tm->t->kernel == id && tm->used < tm->t->per_call) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, tm->t->start[tm->used],
                          tm->t->stop[tm->used], 0, args...);
    tm->used++;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
  }
}

// Timing never fails a solve: a pair whose duration cannot be read is skipped.
static void accumulate(pod2g_timer *t, int used) {
  for (int i = 0; i < used; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(t->stop[i]) != hipSuccess ||
        hipEventElapsedTime(&ms, t->start[i], t->stop[i]) != hipSuccess) {
      (void)hipGetLastError();   // clear the sticky error
      continue;
    }
    t->total_ms += ms;
    t->launches += 1;
  }
}

struct Layout {
  size_t st, ec, part, bpart, vec, vec32, flags, info, arr, total;
  int bgrid;
};

constexpr int BGRID_DEFAULT = 512;    // workgroups of the batched restriction
constexpr int BGRID_MAX = 2048;       // largest the tuner tries (workspace is sized for it)
constexpr long long FUSE_DIR_MAX = 1ll << 20;   // rows x instances with the fused update
// consumer-side sums while (row workgroups x instances) x partials stays
// below this (the partial loads every consumer workgroup repeats)
constexpr long long CONS_MAX = 1ll << 21;

static int batched_grid(int n, int cap) {
  const int nb = ceil_div(n, NT);
  return nb < cap ? nb : cap;
}

static Layout layout(int n, int batch, int k, int precision) {
  const int nb = ceil_div(n, NT);
  const int ps = k > 4 ? k : 4;   // slots 0..3 at least (SLOT_RHO, SLOT_GAMMA)
  Layout L;
  size_t o = 0;
  L.st = o;    o += align256(sizeof(InstState) * (size_t)batch);
  L.ec = o;    o += align256(sizeof(double) * MAXK * (size_t)batch);
  L.part = o;  o += align256(sizeof(double) * (size_t)ps * nb * batch);
  L.bgrid = batched_grid(n, BGRID_DEFAULT);
  L.bpart = o;
  if (precision == POD2G_MIXED && batch >= BATCH_MFMA_MIN && batch <= MAXB && k > 0)
    o += align256(sizeof(double) * (size_t)(batched_grid(n, BGRID_MAX) + 1) * k * batch);
  L.flags = o; o += align256(sizeof(int) * (size_t)batch);
  L.info = o;  o += align256(sizeof(pod2g_slot_info) * (size_t)batch);
  L.arr = o;   o += sizeof(Arrival) * NSITE * (size_t)batch;
  L.vec = o;   o += 8 * align256(sizeof(double) * (size_t)n * batch);   // r p0 p1 q s xa xb r_alt
  L.vec32 = o;
  if (precision == POD2G_MIXED) o += 2 * align256(sizeof(float) * (size_t)n * batch);  // b32, rbuf
  L.total = o;
  return L;
}

// dynamic LDS of the node-wise kernels: the staged neighbourhood of x
template <typename T>
static unsigned xlds(const Ctx &c) {
  return c.xwin ? (unsigned)(sizeof(T) * (size_t)(NT + 2 * c.xwin) * (c.n / c.nn)) : 0u;
}

template <int TJ, int TB, int GRP>
static void launch_ptr_b_g(const Ctx &c, const float *R, hipStream_t stream) {
  if (c.n % 4 == 0)
    hipLaunchKernelGGL((k_ptr_b<TJ, TB, true, GRP>), dim3(c.bgrid), dim3(NT), 0, stream, c, R);
  else
    hipLaunchKernelGGL((k_ptr_b<TJ, TB, false, GRP>), dim3(c.bgrid), dim3(NT), 0, stream, c, R);
}

template <int TJ, int TB>
static void launch_ptr_b_t(const Ctx &c, const float *R, hipStream_t stream) {
  if (c.ptr_grp == 1) launch_ptr_b_g<TJ, TB, 1>(c, R, stream);
  else if (c.ptr_grp == 4) launch_ptr_b_g<TJ, TB, 4>(c, R, stream);
  else launch_ptr_b_g<TJ, TB, 2>(c, R, stream);
}

// the batched restriction with as many basis and batch tiles as k and the
// batch need (k <= 64, 4 <= batch <= 32)
static void launch_ptr_b(const Ctx &c, const float *R, hipStream_t stream) {
  const int tj = (c.k + 15) / 16, tb = (c.batch + 15) / 16;
  switch (tj * 2 + tb - 1) {
    case 2: launch_ptr_b_t<1, 1>(c, R, stream); break;
    case 3: launch_ptr_b_t<1, 2>(c, R, stream); break;
    case 4: launch_ptr_b_t<2, 1>(c, R, stream); break;
    case 5: launch_ptr_b_t<2, 2>(c, R, stream); break;
    case 6: launch_ptr_b_t<3, 1>(c, R, stream); break;
    case 7: launch_ptr_b_t<3, 2>(c, R, stream); break;
    case 8: launch_ptr_b_t<4, 1>(c, R, stream); break;
    default: launch_ptr_b_t<4, 2>(c, R, stream); break;
  }
}

// 2D: stage x around each node block in LDS when the window fits in 48 KB
// at FP64; 3D neighbourhoods span two node planes, which do not fit.
constexpr size_t XWIN_LDS_MAX = 48 * 1024;
static int choose_xwin(const pod2g_pattern *pat) {
  if (pat->mesh.dim != 2) return 0;
  const int w = pat->mesh.N + 1;
  return sizeof(double) * (size_t)(NT + 2 * w) * 2 <= XWIN_LDS_MAX ? w : 0;
}

// Instances per group of the node-wise block order: the largest divisor of
// the batch that is at most IGROUP_MAX.
constexpr int IGROUP_MAX = 1;
static int default_igroup(int batch) {
  int g = IGROUP_MAX;
  while (g > 1 && batch % g) --g;
  return g;
}

static void fill_ctx(Ctx &c, const pod2g_pattern *pat, const double *vals, int batch,
                     const pod2g_prec *prec, const double *f, double *u, void *work) {
  memset(&c, 0, sizeof(c));
  const int n = pat->n;
  const int k = prec ? prec->k : 0;
  const int precision = prec ? prec->precision : POD2G_FP64;
  Layout Lo = layout(n, batch, k, precision);
  char *w = (char *)work;
  c.n = n;
  c.nn = pat->n_nodes;
  c.k = k;
  c.batch = batch;
  c.nb = ceil_div(n, NT);
  c.nbn = ceil_div(pat->n_nodes, NT);
  c.N = pat->mesh.N;
  c.xwin = choose_xwin(pat);
  c.igroup = default_igroup(batch);
  c.fuse_dir = (long long)n * batch <= FUSE_DIR_MAX;
  c.cons = (long long)c.nb * batch * c.nbn <= CONS_MAX;
  c.fuse_upd = (long long)n * batch <= FUSE_DIR_MAX;
  c.ptr_grp = PTR_GRP;
  c.ps = k > 4 ? k : 4;   // as in layout()
  c.vstride = pat->nvals;
  c.colblk = pat->colblk;
  c.vals = vals;
  c.f = f;
  c.u = u;
  c.st = (InstState *)(w + Lo.st);
  c.ec = (double *)(w + Lo.ec);
  c.part = (double *)(w + Lo.part);
  c.bpart = (double *)(w + Lo.bpart);
  c.bgrid = Lo.bgrid;
  c.info = (pod2g_slot_info *)(w + Lo.info);
  c.arr = (Arrival *)(w + Lo.arr);
  const size_t vb = align256(sizeof(double) * (size_t)n * batch);
  c.r = (double *)(w + Lo.vec);
  c.p0 = (double *)(w + Lo.vec + vb);
  c.p1 = (double *)(w + Lo.vec + 2 * vb);
  c.q = (double *)(w + Lo.vec + 3 * vb);
  c.s = (double *)(w + Lo.vec + 4 * vb);
  c.xa = (void *)(w + Lo.vec + 5 * vb);
  c.xb = (void *)(w + Lo.vec + 6 * vb);
  c.r_alt = (double *)(w + Lo.vec + 7 * vb);
  c.b32 = precision == POD2G_MIXED ? (void *)(w + Lo.vec32) : nullptr;
  c.rbuf = precision == POD2G_MIXED
               ? (float *)(w + Lo.vec32 + align256(sizeof(float) * (size_t)n * batch))
               : nullptr;
  c.mixed = precision == POD2G_MIXED;
  if (prec) {
    c.omega = prec->omega;
    c.Linv = prec->Linv;
    c.KP32 = prec->KP32;
    c.KP = prec->KP;
    if (precision == POD2G_MIXED) {
      c.svals = prec->vals32;
      c.sdinv = prec->dinv32;
      c.sP = prec->P32;
    } else {
      c.svals = prec->vals;
      c.sdinv = prec->dinv;
      c.sP = prec->P;
    }
  }
}

// dynamic LDS of the restriction: the k x k inverse factor
static unsigned lds_kk(const Ctx &c) { return (unsigned)(sizeof(double) * c.k * c.k); }

// The cycle's right-hand side as the host sees it (FP64 r or FP32 b32).
template <typename T>
static const T *cycle_rhs_host(const Ctx &c) {
  return sizeof(T) == 8 ? (const T *)c.r : (const T *)c.b32;
}

template <typename T>
static bool batched_products(const Ctx &c) {
  return sizeof(T) == 4 && c.batch >= BATCH_MFMA_MIN && c.batch <= MAXB;
}

// The cycle s = B r on the instances that are not done.  Assumes xa holds
// the first pre-relaxation sweep when nu_pre >= 1 (made by the producer of
// r).  With want_dot the last kernel also forms rho and beta.
template <int DIM, typename T>
static void launch_cycle(const Ctx &c, const pod2g_prec *pr, hipStream_t stream, int want_dot,
                         Tm *tm, int pre2_done) {
  dim3 grid(c.nb, c.batch), gridn(c.nbn, c.batch), blk(NT);
  T *xa = (T *)c.xa, *xb = (T *)c.xb;
  // pre2_done: the first two pre-relaxation sweeps are done, x2 in xb
  T *cur = pre2_done ? xb : xa, *oth = pre2_done ? xa : xb;
  const bool have_x = pr->nu_pre >= 1;
  int post_done = 0;   // post-relaxation sweeps already applied
  for (int i = pre2_done ? 2 : 1; i < pr->nu_pre; ++i) {
    launch(tm, POD2G_TK_SWEEP, k_sweep<DIM, T, false>, gridn, blk, xlds<T>(c), stream, c, (const T *)cur, oth, 0);
    T *t = cur; cur = oth; oth = t;
  }
  bool have = have_x;
  if (c.k > 0 && batched_products<T>(c)) {
    // shared basis, many instances: one MFMA contraction over the batch
    if (have) {
      launch(tm, POD2G_TK_RESTRICT, k_resid32<DIM>, gridn, blk, xlds<float>(c), stream, c, (const float *)cur);
      launch_ptr_b(c, (const float *)c.rbuf, stream);
    } else {
      // x = 0: the residual is the cycle input itself
      launch_ptr_b(c, (const float *)c.b32, stream);
    }
    hipLaunchKernelGGL(k_ptr_sum, dim3(ceil_div((long long)c.k * c.batch * PTR_TPO, NT)), blk, 0,
                       stream, c);
    hipLaunchKernelGGL(k_coarse_b, dim3(c.batch), blk, 0, stream, c);
    // with K P at hand, the first post-sweep comes from the restricted residual
    const float *rp = nullptr;
    if (c.KP32 && pr->nu_post >= 1) rp = have ? (const float *)c.rbuf : (const float *)c.b32;
    launch(tm, POD2G_TK_PROLONG, k_prolong_b, dim3(c.nb), blk, 0, stream, c,
           have ? (const float *)cur : (const float *)nullptr, (float *)oth, rp);
    T *t = cur; cur = oth; oth = t;
    have = true;
    if (rp) post_done = 1;
  } else if (c.k > 0) {
    // with K P at hand the first post-sweep comes from r' (saved by the
    // restriction: q is free during the cycle, rbuf holds FP32)
    const T *kp = sizeof(T) == 8 ? (const T *)c.KP : (const T *)c.KP32;
    T *rsave = nullptr;
    const T *rp = nullptr;
    if (kp && pr->nu_post >= 1) {
      rsave = sizeof(T) == 8 ? (T *)c.q : (T *)c.rbuf;
      rp = have ? (const T *)rsave : cycle_rhs_host<T>(c);
      if (!have) rsave = nullptr;
    }
    if (have)
      launch(tm, POD2G_TK_RESTRICT, k_restrict<DIM, T, false>, grid, blk, lds_kk(c), stream, c,
             (const T *)cur, rsave);
    else
      launch(tm, POD2G_TK_RESTRICT, k_restrict<DIM, T, true>, grid, blk, lds_kk(c), stream, c,
             (const T *)nullptr, (T *)nullptr);
    launch(tm, POD2G_TK_PROLONG, k_prolong<T>, grid, blk, 0, stream, c,
           have ? (const T *)cur : (const T *)nullptr, oth, rp, rp ? kp : (const T *)nullptr);
    T *t = cur; cur = oth; oth = t;
    have = true;
    if (rp) post_done = 1;
  }
  if (pr->nu_post >= 1 && !have) {
    // x = 0 so the first post sweep is omega D^-1 b: reuse the zero-input path
    hipLaunchKernelGGL((k_cyc_first<T>), dim3(c.nb, c.batch), blk, 0, stream, c, 1);
    cur = xa; oth = xb;
    have = true;
    for (int i = 1; i < pr->nu_post; ++i) {
      const bool fin = (i == pr->nu_post - 1);
      if (fin)
        hipLaunchKernelGGL((k_sweep<DIM, T, true>), gridn, blk, xlds<T>(c), stream, c, cur, oth, want_dot);
      else
        hipLaunchKernelGGL((k_sweep<DIM, T, false>), gridn, blk, xlds<T>(c), stream, c, cur, oth, 0);
      T *t = cur; cur = oth; oth = t;
    }
    if (pr->nu_post == 1) hipLaunchKernelGGL((k_finalize<DIM, T>), gridn, blk, 0, stream, c, cur, want_dot);
    return;
  }
  for (int i = post_done; i < pr->nu_post; ++i) {
    const bool fin = (i == pr->nu_post - 1);
    if (fin)
      launch(tm, POD2G_TK_SWEEP_FINAL, k_sweep<DIM, T, true>, gridn, blk, xlds<T>(c), stream, c, (const T *)cur, oth,
             want_dot);
    else
      launch(tm, POD2G_TK_SWEEP, k_sweep<DIM, T, false>, gridn, blk, xlds<T>(c), stream, c, (const T *)cur, oth, 0);
    T *t = cur; cur = oth; oth = t;
  }
  if (pr->nu_post == post_done)
    hipLaunchKernelGGL((k_finalize<DIM, T>), gridn, blk, 0, stream, c, have ? (const T *)cur : (const T *)nullptr, want_dot);
}

// nsweeps Gauss-Seidel sweeps in place on x: colours in turn (reversed
// for backward sweeps).
template <int DIM, typename T>
static void gs_sweeps(const Ctx &c, const T *rhs, T *x, int nsweeps, bool backward,
                      hipStream_t stream) {
  constexpr int NC = 1 << DIM;
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int q = 0; q < NC; ++q) {
      const Colour col = colour_of(DIM, c.N, backward ? NC - 1 - q : q);
      const int cnt = col.ni * col.nj * col.nl;
      if (cnt == 0) continue;
      dim3 g(ceil_div(cnt, NT), c.batch);
      if (backward) hipLaunchKernelGGL((k_gs_colour<DIM, T, true>), g, dim3(NT), 0, stream, c, rhs, x, col);
      else hipLaunchKernelGGL((k_gs_colour<DIM, T, false>), g, dim3(NT), 0, stream, c, rhs, x, col);
    }
  }
}

// The cycle with symmetric Gauss-Seidel relaxation: nu_pre forward sweeps
// from x = 0, restriction, coarse solve and prolongation as in the Jacobi
// cycle, nu_post backward sweeps, then s = x / scale with r^T s.
template <int DIM, typename T>
static void launch_cycle_sgs(const Ctx &c, const pod2g_prec *pr, hipStream_t stream, int want_dot,
                             Tm *tm) {
  dim3 grid(c.nb, c.batch), gridn(c.nbn, c.batch), blk(NT);
  T *x = (T *)c.xa, *y = (T *)c.xb;
  const bool have = pr->nu_pre >= 1;
  if (have) {
    hipLaunchKernelGGL(k_zero<T>, dim3(2048), blk, 0, stream, x, (size_t)c.n * c.batch);
    gs_sweeps<DIM, T>(c, nullptr, x, pr->nu_pre, false, stream);
  }
  T *cur = have ? x : nullptr;
  if (c.k > 0) {
    if (batched_products<T>(c)) {
      if (have) {
        launch(tm, POD2G_TK_RESTRICT, k_resid32<DIM>, gridn, blk, xlds<float>(c), stream, c, (const float *)x);
        launch_ptr_b(c, (const float *)c.rbuf, stream);
      } else {
        launch_ptr_b(c, (const float *)c.b32, stream);
      }
      hipLaunchKernelGGL(k_ptr_sum, dim3(ceil_div((long long)c.k * c.batch * PTR_TPO, NT)), blk, 0,
                         stream, c);
      hipLaunchKernelGGL(k_coarse_b, dim3(c.batch), blk, 0, stream, c);
      launch(tm, POD2G_TK_PROLONG, k_prolong_b, dim3(c.nb), blk, 0, stream, c, (const float *)cur,
             (float *)y, (const float *)nullptr);
    } else {
      if (have)
        launch(tm, POD2G_TK_RESTRICT, k_restrict<DIM, T, false>, grid, blk, lds_kk(c), stream, c,
               (const T *)x, (T *)nullptr);
      else
        launch(tm, POD2G_TK_RESTRICT, k_restrict<DIM, T, true>, grid, blk, lds_kk(c), stream, c,
               (const T *)nullptr, (T *)nullptr);
      launch(tm, POD2G_TK_PROLONG, k_prolong<T>, grid, blk, 0, stream, c, (const T *)cur, y,
             (const T *)nullptr, (const T *)nullptr);
    }
    cur = y;
  } else if (!have) {
    hipLaunchKernelGGL(k_zero<T>, dim3(2048), blk, 0, stream, x, (size_t)c.n * c.batch);
    cur = x;
  }
  if (pr->nu_post >= 1) gs_sweeps<DIM, T>(c, nullptr, cur, pr->nu_post, true, stream);
  hipLaunchKernelGGL((k_finalize<DIM, T>), gridn, blk, 0, stream, c, (const T *)cur, want_dot);
}

template <int DIM>
static void launch_cycle_any(const Ctx &c, const pod2g_prec *pr, hipStream_t stream, int want_dot,
                             Tm *tm, int pre2_done = 0) {
  if (pr->smoother == POD2G_SMOOTHER_SGS) {
    if (pr->precision == POD2G_MIXED) launch_cycle_sgs<DIM, float>(c, pr, stream, want_dot, tm);
    else launch_cycle_sgs<DIM, double>(c, pr, stream, want_dot, tm);
    return;
  }
  if (pr->precision == POD2G_MIXED) launch_cycle<DIM, float>(c, pr, stream, want_dot, tm, pre2_done);
  else launch_cycle<DIM, double>(c, pr, stream, want_dot, tm, pre2_done);
}

template <int DIM>
static void launch_first(const Ctx &c, const pod2g_prec *pr, hipStream_t stream) {
  const int wx = pr->nu_pre >= 1 && pr->smoother == POD2G_SMOOTHER_JACOBI;
  dim3 grid(c.nb, c.batch);
  if (pr->precision == POD2G_MIXED) hipLaunchKernelGGL((k_cyc_first<float>), grid, dim3(NT), 0, stream, c, wx);
  else if (wx) hipLaunchKernelGGL((k_cyc_first<double>), grid, dim3(NT), 0, stream, c, wx);
}

// One PCG iteration.  Iterations alternate the two direction buffers
// (parity 0 reads p0 and writes p1), so chunks have an even length.
template <int DIM>
static void launch_iteration(const Ctx &c, const pod2g_prec *pr, hipStream_t stream, Tm *tm,
                             int parity) {
  dim3 grid(c.nb, c.batch), gridn(c.nbn, c.batch), blk(NT);
  const double *pold = parity ? c.p1 : c.p0;
  double *pnew = parity ? c.p0 : c.p1;
  const double *sdir = pr ? (const double *)c.s : (const double *)c.r;
  // small problems are launch-bound: fold the direction update into the
  // SpMV; large ones are bandwidth-bound: a second gathered vector costs
  // more than one elementwise pass
  // with a preconditioner, rho = r^T s is finished from the cycle's partials
  const int cons = pr ? 1 : 0;
  if (c.fuse_dir) {
    launch(tm, POD2G_TK_SPMV_PQ, k_spmv_pq<DIM, true>, gridn, blk, xlds<double>(c), stream, c, sdir, pold,
           pnew, cons);
  } else {
    hipLaunchKernelGGL(k_pdir, grid, blk, 0, stream, c, sdir, pold, pnew, cons);
    launch(tm, POD2G_TK_SPMV_PQ, k_spmv_pq<DIM, false>, gridn, blk, xlds<double>(c), stream, c, sdir, pold,
           pnew, cons);
  }
  if (pr) {
    const int mode = pr->nu_pre >= 1 && pr->smoother == POD2G_SMOOTHER_JACOBI ? 1 : 2;
    const int fuse = mode == 1 && pr->nu_pre >= 2 && c.fuse_upd;
    if (fuse) {
      // the residual alternates between r (even iterations read it) and
      // r_alt; chunks have an even number of iterations, so it is back in
      // r at the end of each, as every other kernel expects
      const double *rin = parity ? c.r_alt : c.r;
      double *rout = parity ? c.r : c.r_alt;
      if (pr->precision == POD2G_MIXED)
        launch(tm, POD2G_TK_UPDATE, k_update_sweep<DIM, float>, gridn, blk, 0, stream, c,
               (const double *)pnew, rin, rout, (float *)c.xb);
      else
        launch(tm, POD2G_TK_UPDATE, k_update_sweep<DIM, double>, gridn, blk, 0, stream, c,
               (const double *)pnew, rin, rout, (double *)c.xb);
      Ctx cc = c;
      cc.r = rout;
      launch_cycle_any<DIM>(cc, pr, stream, 1, tm, 1);
    } else {
      if (pr->precision == POD2G_MIXED)
        launch(tm, POD2G_TK_UPDATE, k_update<float>, grid, blk, 0, stream, c, mode, (const double *)pnew);
      else
        launch(tm, POD2G_TK_UPDATE, k_update<double>, grid, blk, 0, stream, c, mode, (const double *)pnew);
      launch_cycle_any<DIM>(c, pr, stream, 1, tm);
    }
  } else {
    launch(tm, POD2G_TK_UPDATE, k_update<double>, grid, blk, 0, stream, c, 0, (const double *)pnew);
  }
}

static int read_states(const Ctx &c, std::vector<InstState> &h, hipStream_t stream) {
  h.resize(c.batch);
  POD2G_HIP_CHECK(hipMemcpyAsync(h.data(), c.st, sizeof(InstState) * c.batch,
                                 hipMemcpyDeviceToHost, stream));
  POD2G_HIP_CHECK(hipStreamSynchronize(stream));
  return POD2G_OK;
}

}  // namespace pod2g

// A captured chunk of PCG iterations on fixed buffers (see pcg_plan_create).
struct pod2g_plan {
  pod2g::Ctx c;
  pod2g_pattern pat;
  pod2g_prec prec;
  bool has_prec;
  int chunk;
  hipGraph_t graph;
  hipGraphExec_t exec;
  pod2g_timer *timer;
};

// Slot groups advanced together by one captured graph per step.
struct pod2g_server {
  struct Group {
    pod2g::Ctx c;
    pod2g_prec prec;
    int dim;
    size_t info_off;          // first slot of the group in the info array
    hipGraph_t graph;         // this group's step alone (pod2g_serve_step_group)
    hipGraphExec_t exec;
    // the step of the first pre_n[i] slots only (pod2g_serve_step_prefix),
    // for prefixes 4, 8, 16, ... below the group's slot count
    std::vector<int> pre_n;
    std::vector<hipGraph_t> pre_graph;
    std::vector<hipGraphExec_t> pre_exec;
  };
  std::vector<Group> groups;
  int chunk, slots;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace pod2g {

template <int DIM>
static int pcg_run(Ctx &c, const pod2g_prec *pr, double rtol, int maxit, int beta,
                   int *iters_h, double *relres_h, int *status_h, pod2g_timer *timer,
                   pod2g_plan *plan, hipStream_t stream) {
  dim3 grid(c.nb, c.batch), blk(NT);
  hipLaunchKernelGGL(k_state_init, dim3(ceil_div(c.batch, 64)), dim3(64), 0, stream, c.st, c.arr, c.batch,
                     rtol, maxit, beta, pr ? (const int *)pr->status : (const int *)nullptr);
  hipLaunchKernelGGL(k_init<DIM>, grid, blk, 0, stream, c, pr ? 1 : 0);
  // s = B r and rho; the restart flag makes beta = 0, so the next
  // iteration's direction is p = s (p = r without a preconditioner)
  auto start_cycle = [&]() {
    if (pr) {
      launch_first<DIM>(c, pr, stream);
      launch_cycle_any<DIM>(c, pr, stream, 1, nullptr);
    }
  };
  start_cycle();
  POD2G_HIP_CHECK(hipGetLastError());
  std::vector<InstState> h;
  std::vector<int> flags(c.batch);
  Layout Lo = layout(c.n, c.batch, c.k, pr ? pr->precision : POD2G_FP64);
  int *flags_d = (int *)((char *)c.st - Lo.st + Lo.flags);
  int chunk = plan ? plan->chunk : 4;
  int nchunk = 0;       // chunks launched since the last (re)start
  int launched = 0;     // iterations launched since the last (re)start
  for (int guard = 0; guard < 10000000; ++guard) {
    // the second chunk of a solve is the timed one: caches are warm and no
    // instance can have converged before it unless the solve is very short
    const bool timed = timer && nchunk == 1;
    Tm tm = {timer, 0};
    if (plan && !timed) {
      POD2G_HIP_CHECK(hipGraphLaunch(plan->exec, stream));
    } else {
      for (int i = 0; i < chunk; ++i) launch_iteration<DIM>(c, pr, stream, timed ? &tm : nullptr, i & 1);
      POD2G_HIP_CHECK(hipGetLastError());
    }
    launched += chunk;
    ++nchunk;
    int st = read_states(c, h, stream);
    if (st) return st;
    if (timed) {
      // count the timed launches only if every instance was live through the chunk
      bool live = true;
      for (int b = 0; b < c.batch; ++b) live = live && h[b].iter >= launched;
      if (live) accumulate(timer, tm.used);
    }
    bool all_done = true;
    for (int b = 0; b < c.batch; ++b) all_done = all_done && h[b].done;
    if (!plan && chunk < 16) chunk *= 2;
    if (!all_done) continue;
    // exit check on the true residual
    hipLaunchKernelGGL(k_true_resid<DIM>, grid, blk, 0, stream, c, 0);
    POD2G_HIP_CHECK(hipGetLastError());
    st = read_states(c, h, stream);
    if (st) return st;
    bool any = false;
    for (int b = 0; b < c.batch; ++b) {
      flags[b] = (h[b].status == POD2G_OK && h[b].iter < maxit && h[b].rr_true > h[b].tol2 &&
                  h[b].iter > 0) ? 1 : 0;
      any = any || flags[b];
    }
    if (!any) break;
    POD2G_HIP_CHECK(hipMemcpyAsync(flags_d, flags.data(), sizeof(int) * c.batch,
                                   hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_replace, grid, blk, 0, stream, c, (const int *)flags_d, pr ? 1 : 0);
    start_cycle();
    if (!plan) chunk = 4;
    nchunk = 0;
    launched = 0;
  }
  int ret = POD2G_OK;
  for (int b = 0; b < c.batch; ++b) {
    int s = h[b].status;
    if (s == POD2G_OK && h[b].rr_true > h[b].tol2) s = POD2G_EMAXIT;
    if (iters_h) iters_h[b] = h[b].iter;
    if (relres_h) relres_h[b] = h[b].ff > 0 ? sqrt(h[b].rr_true / h[b].ff) : 0.0;
    if (status_h) status_h[b] = s;
    if (ret == POD2G_OK && s != POD2G_OK) ret = s;
  }
  return ret;
}

// Standalone two-grid iterations u <- u + B (f - K u) until the residual
// test or the iteration limit (maxit >= 1), in growing chunks.
template <int DIM>
static int stat_run(Ctx &c, const pod2g_prec *pr, double rtol, int maxit, int *iters_h,
                    double *relres_h, int *status_h, hipStream_t stream) {
  dim3 grid(c.nb, c.batch), gridn(c.nbn, c.batch), blk(NT);
  hipLaunchKernelGGL(k_state_init, dim3(ceil_div(c.batch, 64)), dim3(64), 0, stream, c.st, c.arr,
                     c.batch, rtol, maxit, (int)POD2G_BETA_FR, (const int *)pr->status);
  hipLaunchKernelGGL(k_init<DIM>, grid, blk, 0, stream, c, 1);
  POD2G_HIP_CHECK(hipGetLastError());
  std::vector<InstState> h;
  int chunk = 4;
  for (int guard = 0; guard < 10000000; ++guard) {
    for (int i = 0; i < chunk; ++i) {
      launch_first<DIM>(c, pr, stream);
      launch_cycle_any<DIM>(c, pr, stream, 0, nullptr);
      hipLaunchKernelGGL(k_stat_update, grid, blk, 0, stream, c);
      hipLaunchKernelGGL(k_stat_resid<DIM>, gridn, blk, xlds<double>(c), stream, c);
    }
    POD2G_HIP_CHECK(hipGetLastError());
    int st = read_states(c, h, stream);
    if (st) return st;
    bool all_done = true;
    for (int b = 0; b < c.batch; ++b) all_done = all_done && h[b].done;
    if (all_done) break;
    if (chunk < 16) chunk *= 2;
  }
  int ret = POD2G_OK;
  for (int b = 0; b < c.batch; ++b) {
    const int s = h[b].status;
    if (iters_h) iters_h[b] = h[b].iter;
    if (relres_h) relres_h[b] = h[b].ff > 0 ? sqrt(h[b].rr / h[b].ff) : 0.0;
    if (status_h) status_h[b] = s;
    if (ret == POD2G_OK && s != POD2G_OK) ret = s;
  }
  return ret;
}

// ---------------------------------------------------------------------------
// single kernels: y = K x and damped-Jacobi sweeps
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(NT) k_spmv(int n, int nn, int nb, long long vstride,
                                             const int *__restrict__ colblk,
                                             const double *__restrict__ vals,
                                             const double *__restrict__ x, double *__restrict__ y) {
  const int b = blockIdx.y;
  const int row = xcd_block(blockIdx.x, nb) * NT + threadIdx.x;
  if (row >= n) return;
  const size_t off = (size_t)b * n;
  y[off + row] = row_dot<DIM>(colblk, vals + (size_t)b * vstride, x + off, row, row / DIM, n, nn);
}

__global__ void k_mark_begin() {}
__global__ void k_mark_end() {}

}  // namespace pod2g

using namespace pod2g;

extern "C" {

int pod2g_mark(int which, hipStream_t stream) {
  if (which == 0) hipLaunchKernelGGL(k_mark_begin, dim3(1), dim3(1), 0, stream);
  else if (which == 1) hipLaunchKernelGGL(k_mark_end, dim3(1), dim3(1), 0, stream);
  else return POD2G_EINVAL;
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

const char *pod2g_strerror(int s) {
  switch (s) {
    case POD2G_OK: return "ok";
    case POD2G_EINVAL: return "invalid argument";
    case POD2G_ESIZE: return "workspace too small";
    case POD2G_EHIP: return "HIP runtime error";
    case POD2G_ENOTSPD: return "coarse matrix P^T K P is not positive definite";
    case POD2G_ESMOOTHER: return "damped-Jacobi smoother diverges: omega * lambda_max(D^-1 K) >= 2";
    case POD2G_EMAXIT: return "iteration limit reached";
    case POD2G_EBREAKDOWN: return "CG breakdown: p^T K p <= 0 or r^T s <= 0";
    case POD2G_ENAN: return "non-finite value";
    default: return "unknown status";
  }
}

size_t pcg_solve_bytes(const pod2g_pattern *pat, int batch, int k, int precision) {
  if (!pat || batch < 1 || k < 0 || k > MAXK) return 0;
  return layout(pat->n, batch, k, precision).total;
}

size_t pod2g_apply_bytes(const pod2g_prec *prec) {
  if (!prec) return 0;
  return layout(prec->pat.n, prec->batch, prec->k, prec->precision).total;
}

static int check_prec(const pod2g_prec *pr) {
  if (pr->k < 0 || pr->k > MAXK || pr->batch < 1 || pr->batch > 65535) return POD2G_EINVAL;
  if (pr->nu_pre < 0 || pr->nu_post < 0 || pr->nu_pre > 64 || pr->nu_post > 64) return POD2G_EINVAL;
  if (pr->precision == POD2G_MIXED && (!pr->vals32 || !pr->dinv32 || (pr->k > 0 && !pr->P32)))
    return POD2G_EINVAL;
  if (pr->k > 0 && (!pr->P || !pr->L || !pr->Linv)) return POD2G_EINVAL;
  return POD2G_OK;
}

static int check_solve_args(const pod2g_pattern *pat, const double *vals, int batch,
                            const pod2g_prec *prec, const double *f, double *u, int beta,
                            void *work, size_t bytes) {
  if (!pat || !vals || !f || !u || !work || batch < 1 || batch > 65535) return POD2G_EINVAL;
  if (beta != POD2G_BETA_FR && beta != POD2G_BETA_PR) return POD2G_EINVAL;
  if (prec) {
    if (check_prec(prec)) return POD2G_EINVAL;
    if (prec->batch != batch || prec->pat.n != pat->n || prec->vals != vals) return POD2G_EINVAL;
  }
  const int k = prec ? prec->k : 0;
  if (bytes < pcg_solve_bytes(pat, batch, k, prec ? prec->precision : POD2G_FP64)) return POD2G_ESIZE;
  return POD2G_OK;
}

int pcg_solve_timed(const pod2g_pattern *pat, const double *vals, int batch,
                    const pod2g_prec *prec, const double *f, double *u, double rtol, int maxit,
                    int beta, int *iters_h, double *relres_h, int *status_h, void *work,
                    size_t bytes, pod2g_timer *timer, hipStream_t stream) {
  int st = check_solve_args(pat, vals, batch, prec, f, u, beta, work, bytes);
  if (st) return st;
  if (!(rtol >= 0.0) || maxit < 0) return POD2G_EINVAL;
  Ctx c;
  fill_ctx(c, pat, vals, batch, prec, f, u, work);
  if (pat->mesh.dim == 2)
    return pcg_run<2>(c, prec, rtol, maxit, beta, iters_h, relres_h, status_h, timer, nullptr, stream);
  return pcg_run<3>(c, prec, rtol, maxit, beta, iters_h, relres_h, status_h, timer, nullptr, stream);
}

int pod2g_stationary_solve(const pod2g_pattern *pat, const double *vals, int batch,
                           const pod2g_prec *prec, const double *f, double *u, double rtol,
                           int maxit, int *iters_h, double *relres_h, int *status_h, void *work,
                           size_t bytes, hipStream_t stream) {
  if (!prec) return POD2G_EINVAL;
  int st = check_solve_args(pat, vals, batch, prec, f, u, POD2G_BETA_FR, work, bytes);
  if (st) return st;
  if (!(rtol >= 0.0) || maxit < 1) return POD2G_EINVAL;
  Ctx c;
  fill_ctx(c, pat, vals, batch, prec, f, u, work);
  if (pat->mesh.dim == 2) return stat_run<2>(c, prec, rtol, maxit, iters_h, relres_h, status_h, stream);
  return stat_run<3>(c, prec, rtol, maxit, iters_h, relres_h, status_h, stream);
}

}  // extern "C"

namespace pod2g {

// Reduced-order solution u = P (P^T K P)^{-1} P^T f.  P^T f: one workgroup
// per basis column, fixed-order sums (four independent accumulators per
// thread, then the block tree).
__global__ void __launch_bounds__(NT) k_rom_restrict(int n, const double *__restrict__ P,
                                                     const double *__restrict__ f,
                                                     double *__restrict__ pf) {
  __shared__ double lds[NWAVE];
  const double *Pj = P + (size_t)blockIdx.x * n;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * NT < n; i += 4 * NT) {
    a0 += Pj[i] * f[i];
    a1 += Pj[i + NT] * f[i + NT];
    a2 += Pj[i + 2 * NT] * f[i + 2 * NT];
    a3 += Pj[i + 3 * NT] * f[i + 3 * NT];
  }
  for (; i < n; i += NT) a0 += Pj[i] * f[i];
  const double v = block_sum((a0 + a1) + (a2 + a3), lds);
  if (threadIdx.x == 0) pf[blockIdx.x] = v;
}

// e_b = Linv_b^T (Linv_b P^T f), one workgroup per instance.
__global__ void __launch_bounds__(NT) k_rom_coarse(int k, const double *__restrict__ Linv,
                                                   const double *__restrict__ pf,
                                                   double *__restrict__ e) {
  __shared__ double y[MAXK];
  const int b = blockIdx.x, t = threadIdx.x;
  const double *Li = Linv + (size_t)b * k * k;
  if (t < k) {
    double v = 0.0;
    for (int j = 0; j <= t; ++j) v += Li[t * k + j] * pf[j];
    y[t] = v;
  }
  __syncthreads();
  if (t < k) {
    double v = 0.0;
    for (int j = t; j < k; ++j) v += Li[j * k + t] * y[j];
    e[(size_t)b * MAXK + t] = v;
  }
}

// u_b = P e_b.
__global__ void __launch_bounds__(NT) k_rom_prolong(int n, int k, const double *__restrict__ P,
                                                    const double *__restrict__ e,
                                                    double *__restrict__ u) {
  __shared__ double es[MAXK];
  const int b = blockIdx.y;
  if (threadIdx.x < k) es[threadIdx.x] = e[(size_t)b * MAXK + threadIdx.x];
  __syncthreads();
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += P[(size_t)j * n + row] * es[j];
  u[(size_t)b * n + row] = acc;
}

}  // namespace pod2g

extern "C" {

size_t pod2g_rom_bytes(const pod2g_prec *prec) {
  if (!prec || prec->batch < 1) return 0;
  return align256(sizeof(double) * MAXK) + align256(sizeof(double) * MAXK * (size_t)prec->batch);
}

int pod2g_rom_start(const pod2g_prec *prec, const double *f, double *u, void *work, size_t bytes,
                    hipStream_t stream) {
  if (!prec || !f || !u || !work || check_prec(prec)) return POD2G_EINVAL;
  if (prec->k < 1) return POD2G_EINVAL;
  if (bytes < pod2g_rom_bytes(prec)) return POD2G_ESIZE;
  const int n = prec->pat.n, k = prec->k, B = prec->batch;
  double *pf = (double *)work;
  double *e = (double *)((char *)work + align256(sizeof(double) * MAXK));
  hipLaunchKernelGGL(k_rom_restrict, dim3(k), dim3(NT), 0, stream, n, prec->P, f, pf);
  hipLaunchKernelGGL(k_rom_coarse, dim3(B), dim3(NT), 0, stream, k, (const double *)prec->Linv,
                     (const double *)pf, e);
  hipLaunchKernelGGL(k_rom_prolong, dim3(ceil_div(n, NT), B), dim3(NT), 0, stream, n, k, prec->P,
                     (const double *)e, u);
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

int pcg_solve(const pod2g_pattern *pat, const double *vals, int batch, const pod2g_prec *prec,
              const double *f, double *u, double rtol, int maxit, int beta, int *iters_h,
              double *relres_h, int *status_h, void *work, size_t bytes, hipStream_t stream) {
  return pcg_solve_timed(pat, vals, batch, prec, f, u, rtol, maxit, beta, iters_h, relres_h,
                         status_h, work, bytes, nullptr, stream);
}

}  // extern "C"

namespace pod2g {

// (Re)capture the plan's chunk of iterations into its graph.
static int capture_plan(pod2g_plan *pl) {
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  pl->exec = nullptr;
  pl->graph = nullptr;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return POD2G_EHIP;
  const pod2g_prec *pr = pl->has_prec ? &pl->prec : nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    for (int i = 0; i < pl->chunk; ++i) {
      if (pl->pat.mesh.dim == 2) launch_iteration<2>(pl->c, pr, cs, nullptr, i & 1);
      else launch_iteration<3>(pl->c, pr, cs, nullptr, i & 1);
    }
    ok = hipStreamEndCapture(cs, &pl->graph) == hipSuccess;
  }
  if (ok && hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(pl->graph);
    pl->graph = nullptr;
    ok = false;
  }
  (void)hipStreamDestroy(cs);
  return ok ? POD2G_OK : POD2G_EHIP;
}

// Average time of one PCG iteration with the Ctx's launch parameters: a
// fresh start with rtol = 0 (no instance stops), two warm-up iterations,
// then `trials` timed ones (eager launches).
template <int DIM>
static int time_iterations(Ctx &c, const pod2g_prec *pr, int trials, hipStream_t s, float *ms) {
  dim3 grid(c.nb, c.batch), blk(NT);
  const int beta = pr && pr->precision == POD2G_MIXED ? POD2G_BETA_PR : POD2G_BETA_FR;
  hipLaunchKernelGGL(k_state_init, dim3(ceil_div(c.batch, 64)), dim3(64), 0, s, c.st, c.arr, c.batch,
                     0.0, 1 << 30, beta, pr ? (const int *)pr->status : (const int *)nullptr);
  hipLaunchKernelGGL(k_init<DIM>, grid, blk, 0, s, c, pr ? 1 : 0);
  if (pr) {
    launch_first<DIM>(c, pr, s);
    launch_cycle_any<DIM>(c, pr, s, 1, nullptr);
  }
  launch_iteration<DIM>(c, pr, s, nullptr, 0);
  launch_iteration<DIM>(c, pr, s, nullptr, 1);
  hipEvent_t e0, e1;
  POD2G_HIP_CHECK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return POD2G_EHIP; }
  int st = POD2G_OK;
  if (hipEventRecord(e0, s) != hipSuccess) st = POD2G_EHIP;
  for (int i = 0; st == POD2G_OK && i < trials; ++i) launch_iteration<DIM>(c, pr, s, nullptr, i & 1);
  if (st == POD2G_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                         hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    st = POD2G_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == POD2G_OK) *ms /= trials;
  return st;
}

}  // namespace pod2g

extern "C" {

int pcg_plan_tune(pod2g_plan *pl, int trials, pod2g_tuning *out, hipStream_t stream) {
  if (!pl || trials < 2 || trials > 1000) return POD2G_EINVAL;
  Ctx &c = pl->c;
  const pod2g_prec *pr = pl->has_prec ? &pl->prec : nullptr;
  auto measure = [&](float *ms) {
    return pl->pat.mesh.dim == 2 ? time_iterations<2>(c, pr, trials, stream, ms)
                                 : time_iterations<3>(c, pr, trials, stream, ms);
  };
  float best = 0.f;
  int st = measure(&best);
  if (st) return st;
  // one parameter at a time, keeping the best value of each
  std::vector<int> grids;
  if (pr && pr->precision == POD2G_MIXED && batched_products<float>(c) && c.k > 0) {
    const int cap = batched_grid(c.n, BGRID_MAX);
    for (int g : {256, 512, 1024, 2048})
      if (g <= cap) grids.push_back(g);
  }
  for (int g : grids) {
    if (g == c.bgrid) continue;
    const int keep = c.bgrid;
    c.bgrid = g;
    float ms;
    if ((st = measure(&ms))) return st;
    if (ms < best) best = ms;
    else c.bgrid = keep;
  }
  {
    const int keep = c.fuse_dir;
    c.fuse_dir = !keep;
    float ms;
    if ((st = measure(&ms))) return st;
    if (ms < best) best = ms;
    else c.fuse_dir = keep;
  }
  if (pr && pr->nu_pre >= 2 && pr->smoother == POD2G_SMOOTHER_JACOBI) {
    // the vector update fused with the second pre-relaxation sweep, or not
    const int keep = c.fuse_upd;
    c.fuse_upd = !keep;
    float ms;
    if ((st = measure(&ms))) return st;
    if (ms < best) best = ms;
    else c.fuse_upd = keep;
  }
  {
    // the scalar sums finished by their consumers, or by the producers
    const int keep = c.cons;
    c.cons = !keep;
    float ms;
    if ((st = measure(&ms))) return st;
    if (ms < best) best = ms;
    else c.cons = keep;
  }
  {
    // the neighbourhood of each node block staged in LDS, or gathers from L2
    const int keep = c.xwin;
    c.xwin = keep ? 0 : choose_xwin(&pl->pat);
    if (c.xwin != keep) {
      float ms;
      if ((st = measure(&ms))) return st;
      if (ms < best) best = ms;
      else c.xwin = keep;
    }
  }
  if (!grids.empty()) {
    // row groups of the batched restriction loaded together
    for (int g : {1, 2, 4}) {
      if (g == c.ptr_grp) continue;
      const int keep = c.ptr_grp;
      c.ptr_grp = g;
      float ms;
      if ((st = measure(&ms))) return st;
      if (ms < best) best = ms;
      else c.ptr_grp = keep;
    }
  }
  for (int g : {1, 2, 4, 8}) {
    if (g == c.igroup || c.batch % g) continue;
    const int keep = c.igroup;
    c.igroup = g;
    float ms;
    if ((st = measure(&ms))) return st;
    if (ms < best) best = ms;
    else c.igroup = keep;
  }
  if ((st = capture_plan(pl))) return st;
  if (out) {
    out->bgrid = c.bgrid;
    out->fuse_dir = c.fuse_dir;
    out->igroup = c.igroup;
    out->xwin = c.xwin;
    out->cons = c.cons;
    out->fuse_upd = c.fuse_upd;
    out->ptr_grp = c.ptr_grp;
    out->ms_per_iteration = best;
  }
  return POD2G_OK;
}

int pcg_plan_configure(pod2g_plan *pl, const pod2g_tuning *cfg) {
  if (!pl || !cfg) return POD2G_EINVAL;
  Ctx &c = pl->c;
  const int gmax = batched_grid(c.n, BGRID_MAX);
  if (cfg->bgrid < 1 || cfg->bgrid > gmax) return POD2G_EINVAL;
  if ((cfg->fuse_dir | cfg->cons | cfg->fuse_upd) & ~1) return POD2G_EINVAL;
  if (cfg->igroup < 1 || cfg->igroup > 8 || c.batch % cfg->igroup) return POD2G_EINVAL;
  if (cfg->ptr_grp != 1 && cfg->ptr_grp != 2 && cfg->ptr_grp != 4) return POD2G_EINVAL;
  const int xw = cfg->xwin > 0 ? choose_xwin(&pl->pat) : 0;
  if (cfg->xwin < 0 || (cfg->xwin > 0 && xw == 0)) return POD2G_EINVAL;
  const Ctx keep = c;
  c.bgrid = cfg->bgrid;
  c.fuse_dir = cfg->fuse_dir;
  c.igroup = cfg->igroup;
  c.xwin = xw;
  c.cons = cfg->cons;
  c.fuse_upd = cfg->fuse_upd;
  c.ptr_grp = cfg->ptr_grp;
  const int st = capture_plan(pl);
  if (st) c = keep;
  return st;
}

int pcg_plan_config(const pod2g_plan *pl, pod2g_tuning *out) {
  if (!pl || !out) return POD2G_EINVAL;
  out->bgrid = pl->c.bgrid;
  out->fuse_dir = pl->c.fuse_dir;
  out->igroup = pl->c.igroup;
  out->xwin = pl->c.xwin;
  out->cons = pl->c.cons;
  out->fuse_upd = pl->c.fuse_upd;
  out->ptr_grp = pl->c.ptr_grp;
  out->ms_per_iteration = 0.f;
  return POD2G_OK;
}

int pcg_plan_create(const pod2g_pattern *pat, const double *vals, int batch, const pod2g_prec *prec,
                    const double *f, double *u, int chunk, void *work, size_t bytes,
                    pod2g_timer *timer, pod2g_plan **out) {
  if (!out) return POD2G_EINVAL;
  int st = check_solve_args(pat, vals, batch, prec, f, u, POD2G_BETA_FR, work, bytes);
  if (st) return st;
  if (chunk < 1 || chunk > 256) return POD2G_EINVAL;
  chunk += chunk & 1;   // even: every replay starts on the same direction buffer
  pod2g_plan *pl = new pod2g_plan;
  memset(pl, 0, sizeof(*pl));
  pl->pat = *pat;
  pl->has_prec = prec != nullptr;
  if (prec) pl->prec = *prec;
  pl->chunk = chunk;
  pl->timer = timer;
  fill_ctx(pl->c, pat, vals, batch, prec, f, u, work);
  if (capture_plan(pl) != POD2G_OK) {
    delete pl;
    return POD2G_EHIP;
  }
  *out = pl;
  return POD2G_OK;
}

int pcg_plan_solve(pod2g_plan *pl, double rtol, int maxit, int beta, int *iters_h,
                   double *relres_h, int *status_h, hipStream_t stream) {
  if (!pl || !(rtol >= 0.0) || maxit < 0) return POD2G_EINVAL;
  if (beta != POD2G_BETA_FR && beta != POD2G_BETA_PR) return POD2G_EINVAL;
  const pod2g_prec *pr = pl->has_prec ? &pl->prec : nullptr;
  if (pl->pat.mesh.dim == 2)
    return pcg_run<2>(pl->c, pr, rtol, maxit, beta, iters_h, relres_h, status_h, pl->timer, pl, stream);
  return pcg_run<3>(pl->c, pr, rtol, maxit, beta, iters_h, relres_h, status_h, pl->timer, pl, stream);
}

int pcg_plan_destroy(pod2g_plan *pl) {
  if (!pl) return POD2G_EINVAL;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  delete pl;
  return POD2G_OK;
}

static void serve_group_step(const pod2g_server::Group &g, int chunk, hipStream_t cs) {
  dim3 grid(g.c.nb, g.c.batch), blk(NT);
  if (g.dim == 2) {
    hipLaunchKernelGGL(k_true_resid<2>, grid, blk, 0, cs, g.c, 1);
    for (int i = 0; i < chunk; ++i) launch_iteration<2>(g.c, &g.prec, cs, nullptr, i & 1);
    hipLaunchKernelGGL(k_true_resid<2>, grid, blk, 0, cs, g.c, 1);
  } else {
    hipLaunchKernelGGL(k_true_resid<3>, grid, blk, 0, cs, g.c, 1);
    for (int i = 0; i < chunk; ++i) launch_iteration<3>(g.c, &g.prec, cs, nullptr, i & 1);
    hipLaunchKernelGGL(k_true_resid<3>, grid, blk, 0, cs, g.c, 1);
  }
}

int pod2g_server_create(const pod2g_group *groups, int n_groups, int chunk, pod2g_server **out,
                        hipStream_t stream) {
  if (!out || !groups || n_groups < 1 || n_groups > 64 || chunk < 2 || chunk > 256)
    return POD2G_EINVAL;
  chunk += chunk & 1;
  pod2g_server *sv = new pod2g_server;
  sv->chunk = chunk;
  sv->slots = 0;
  sv->graph = nullptr;
  sv->exec = nullptr;
  for (int g = 0; g < n_groups; ++g) {
    const pod2g_group &G = groups[g];
    if (!G.prec) { delete sv; return POD2G_EINVAL; }
    const int batch = G.prec->batch;
    int st = check_solve_args(G.pat, G.vals, batch, G.prec, G.f, G.u, POD2G_BETA_FR, G.work, G.bytes);
    if (st) { delete sv; return st; }
    pod2g_server::Group gr;
    gr.prec = *G.prec;
    gr.dim = G.pat->mesh.dim;
    gr.info_off = (size_t)sv->slots;
    gr.graph = nullptr;
    gr.exec = nullptr;
    fill_ctx(gr.c, G.pat, G.vals, batch, G.prec, G.f, G.u, G.work);
    sv->groups.push_back(gr);
    sv->slots += batch;
  }
  for (auto &g : sv->groups)
    hipLaunchKernelGGL(k_serve_free, dim3(ceil_div(g.c.batch, 64)), dim3(64), 0, stream, g.c.st, g.c.arr,
                       g.c.info, g.c.batch);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
    delete sv;
    return POD2G_EHIP;
  }
  // Capture: one branch per group (forked from and joined into the capture
  // stream with events), so the groups' kernels may run side by side and a
  // small class does not wait for a large one's iterations.
  const int G = (int)sv->groups.size();
  std::vector<hipStream_t> bs(G, nullptr);
  std::vector<hipEvent_t> done_ev(G, nullptr);
  hipStream_t cs = nullptr;
  hipEvent_t fork = nullptr;
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
  for (int g = 0; ok && g < G; ++g)
    ok = hipStreamCreateWithFlags(&bs[g], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&done_ev[g], hipEventDisableTiming) == hipSuccess;
  if (ok) ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    bool cap = hipEventRecord(fork, cs) == hipSuccess;
    for (int g = 0; cap && g < G; ++g) {
      cap = hipStreamWaitEvent(bs[g], fork, 0) == hipSuccess;
      if (cap) serve_group_step(sv->groups[g], chunk, bs[g]);
      cap = cap && hipEventRecord(done_ev[g], bs[g]) == hipSuccess &&
            hipStreamWaitEvent(cs, done_ev[g], 0) == hipSuccess;
    }
    const bool ended = hipStreamEndCapture(cs, &sv->graph) == hipSuccess;
    ok = cap && ended;
  }
  if (ok && hipGraphInstantiate(&sv->exec, sv->graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
  // one graph per group as well, for groups stepped at their own pace, and
  // one per slot prefix: the same kernels and launch parameters over the
  // first m slots (m >= 4 keeps the batched products, whose sums per slot
  // do not depend on the batch width, so a slot gets the same bits from any
  // prefix that holds it)
  for (int g = 0; ok && g < G; ++g) {
    auto &gr = sv->groups[g];
    ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (!ok) break;
    serve_group_step(gr, chunk, cs);
    ok = hipStreamEndCapture(cs, &gr.graph) == hipSuccess;
    if (ok && hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
    // (a mixed group wider than the batched products' limit runs per
    // instance, its prefixes would not: no prefixes then)
    const bool same_path = !(gr.prec.precision == POD2G_MIXED && gr.c.batch > MAXB);
    for (int m = BATCH_MFMA_MIN; ok && same_path && m < gr.c.batch; m *= 2) {
      pod2g_server::Group pre = gr;
      pre.c.batch = m;
      hipGraph_t pg = nullptr;
      hipGraphExec_t pe = nullptr;
      ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (!ok) break;
      serve_group_step(pre, chunk, cs);
      ok = hipStreamEndCapture(cs, &pg) == hipSuccess;
      if (ok && hipGraphInstantiate(&pe, pg, nullptr, nullptr, 0) != hipSuccess) ok = false;
      if (pg) {
        gr.pre_n.push_back(m);
        gr.pre_graph.push_back(pg);
        gr.pre_exec.push_back(pe);
      }
    }
  }
  for (int g = 0; g < G; ++g) {
    if (done_ev[g]) (void)hipEventDestroy(done_ev[g]);
    if (bs[g]) (void)hipStreamDestroy(bs[g]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok) {
    pod2g_server_destroy(sv);
    return POD2G_EHIP;
  }
  *out = sv;
  return POD2G_OK;
}

int pod2g_server_admit(pod2g_server *sv, int group, int slot, double rtol, int maxit, int beta,
                       hipStream_t stream) {
  if (!sv || group < 0 || group >= (int)sv->groups.size()) return POD2G_EINVAL;
  const pod2g_server::Group &g = sv->groups[group];
  if (slot < 0 || slot >= g.c.batch || !(rtol >= 0.0) || maxit < 0) return POD2G_EINVAL;
  if (beta != POD2G_BETA_FR && beta != POD2G_BETA_PR) return POD2G_EINVAL;
  hipLaunchKernelGGL(k_serve_admit, dim3(1), dim3(64), 0, stream, g.c.st, g.c.arr, g.c.info, slot, rtol,
                     maxit, beta, (const int *)g.prec.status);
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

int pod2g_serve_step(pod2g_server *sv, pod2g_slot_info *info_h, hipStream_t stream) {
  if (!sv || !info_h) return POD2G_EINVAL;
  POD2G_HIP_CHECK(hipGraphLaunch(sv->exec, stream));
  size_t off = 0;
  for (const auto &g : sv->groups) {
    POD2G_HIP_CHECK(hipMemcpyAsync(info_h + off, g.c.info, sizeof(pod2g_slot_info) * g.c.batch,
                                   hipMemcpyDeviceToHost, stream));
    off += g.c.batch;
  }
  return POD2G_OK;
}

int pod2g_serve_step_group(pod2g_server *sv, int group, pod2g_slot_info *info_h,
                           hipStream_t stream) {
  if (!sv || !info_h || group < 0 || group >= (int)sv->groups.size()) return POD2G_EINVAL;
  const pod2g_server::Group &g = sv->groups[group];
  POD2G_HIP_CHECK(hipGraphLaunch(g.exec, stream));
  POD2G_HIP_CHECK(hipMemcpyAsync(info_h + g.info_off, g.c.info,
                                 sizeof(pod2g_slot_info) * g.c.batch, hipMemcpyDeviceToHost, stream));
  return POD2G_OK;
}

int pod2g_serve_step_prefix(pod2g_server *sv, int group, int nslots, pod2g_slot_info *info_h,
                            hipStream_t stream) {
  if (!sv || !info_h || group < 0 || group >= (int)sv->groups.size()) return POD2G_EINVAL;
  const pod2g_server::Group &g = sv->groups[group];
  if (nslots < 0 || nslots > g.c.batch) return POD2G_EINVAL;
  hipGraphExec_t e = g.exec;
  for (size_t i = 0; i < g.pre_n.size(); ++i)
    if (nslots <= g.pre_n[i] && g.pre_exec[i]) {
      e = g.pre_exec[i];
      break;
    }
  POD2G_HIP_CHECK(hipGraphLaunch(e, stream));
  POD2G_HIP_CHECK(hipMemcpyAsync(info_h + g.info_off, g.c.info,
                                 sizeof(pod2g_slot_info) * g.c.batch, hipMemcpyDeviceToHost, stream));
  return POD2G_OK;
}

int pod2g_stream_create_cus(int cu_first, int cu_count, hipStream_t *out) {
  if (!out || cu_first < 0 || cu_count < 1) return POD2G_EINVAL;
  int dev = 0;
  POD2G_HIP_CHECK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  POD2G_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  const int ncu = prop.multiProcessorCount;
  if (cu_first + cu_count > ncu) return POD2G_EINVAL;
  std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
  for (int cu = cu_first; cu < cu_first + cu_count; ++cu) mask[cu / 32] |= 1u << (cu % 32);
  POD2G_HIP_CHECK(hipExtStreamCreateWithCUMask(out, (uint32_t)mask.size(), mask.data()));
  return POD2G_OK;
}

int pod2g_stream_destroy(hipStream_t s) {
  if (!s) return POD2G_EINVAL;
  POD2G_HIP_CHECK(hipStreamDestroy(s));
  return POD2G_OK;
}

int pod2g_server_slots(const pod2g_server *sv) { return sv ? sv->slots : POD2G_EINVAL; }

int pod2g_server_destroy(pod2g_server *sv) {
  if (!sv) return POD2G_EINVAL;
  for (auto &g : sv->groups) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    for (auto e : g.pre_exec)
      if (e) (void)hipGraphExecDestroy(e);
    for (auto gr : g.pre_graph)
      if (gr) (void)hipGraphDestroy(gr);
  }
  if (sv->exec) (void)hipGraphExecDestroy(sv->exec);
  if (sv->graph) (void)hipGraphDestroy(sv->graph);
  delete sv;
  return POD2G_OK;
}

int pod2g_timer_create(int kernel, int per_call, pod2g_timer *out) {
  if (!out || per_call < 1 || per_call > 4096 || kernel < POD2G_TK_SPMV_PQ || kernel > POD2G_TK_UPDATE)
    return POD2G_EINVAL;
  pod2g_timer t;
  memset(&t, 0, sizeof(t));
  t.kernel = kernel;
  t.per_call = per_call;
  t.start = new hipEvent_t[per_call];
  t.stop = new hipEvent_t[per_call];
  for (int i = 0; i < per_call; ++i) {
    if (hipEventCreate(&t.start[i]) != hipSuccess || hipEventCreate(&t.stop[i]) != hipSuccess) {
      delete[] t.start;
      delete[] t.stop;
      return POD2G_EHIP;
    }
  }
  *out = t;
  return POD2G_OK;
}

int pod2g_timer_reset(pod2g_timer *t) {
  if (!t) return POD2G_EINVAL;
  t->total_ms = 0.0;
  t->launches = 0;
  return POD2G_OK;
}

int pod2g_timer_destroy(pod2g_timer *t) {
  if (!t || !t->start) return POD2G_EINVAL;
  for (int i = 0; i < t->per_call; ++i) {
    (void)hipEventDestroy(t->start[i]);
    (void)hipEventDestroy(t->stop[i]);
  }
  delete[] t->start;
  delete[] t->stop;
  t->start = t->stop = nullptr;
  t->per_call = 0;
  return POD2G_OK;
}

// s = B r: the same kernels as inside PCG, on a scratch state.
__global__ void k_apply_init(InstState *st, Arrival *arr, int batch, const double *sc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  zero_arrivals(arr + (size_t)b * NSITE, NSITE, 0, 1);
  InstState s;
  memset(&s, 0, sizeof(s));
  s.scale = sc ? sc[b] : 1.0;
  s.restart = 1;
  st[b] = s;
}

}  // extern "C"

// One cycle s = B r on the caller's arrays with the workspace `work`
// (arguments already checked).
static int apply_run(const pod2g_prec *prec, const double *r, double *s, void *work,
                     hipStream_t stream) {
  Ctx c;
  fill_ctx(c, &prec->pat, prec->vals, prec->batch, prec, nullptr, nullptr, work);
  // the cycle reads r from c.r and writes c.s; run it on the caller's arrays
  c.r = const_cast<double *>(r);
  c.s = s;
  hipLaunchKernelGGL(k_apply_init, dim3(ceil_div(c.batch, 64)), dim3(64), 0, stream, c.st, c.arr, c.batch,
                     (const double *)nullptr);
  if (prec->pat.mesh.dim == 2) {
    launch_first<2>(c, prec, stream);
    launch_cycle_any<2>(c, prec, stream, 0, nullptr);
  } else {
    launch_first<3>(c, prec, stream);
    launch_cycle_any<3>(c, prec, stream, 0, nullptr);
  }
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

// Scratch of pod2g_apply_noalloc: one array per GPU the library runs on,
// held until the process ends.  On the host its name is only a stand-in:
// host code uses the device address hipGetSymbolAddress gives for the
// current device (kept per device), never the name itself.
static __device__ __align__(256) unsigned char scratch[POD2G_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAXDEV = 64;
static std::mutex scratch_mu;
static void *scratch_ptr[SCRATCH_MAXDEV];

static int scratch_address(void **out) {
  int dev = -1;
  POD2G_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAXDEV) return POD2G_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return POD2G_EHIP;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return POD2G_OK;
}

extern "C" {

int pod2g_apply(const pod2g_prec *prec, const double *r, double *s, void *work, size_t bytes,
                hipStream_t stream) {
  if (!prec || !r || !s || !work) return POD2G_EINVAL;
  if (check_prec(prec)) return POD2G_EINVAL;
  if (bytes < pod2g_apply_bytes(prec)) return POD2G_ESIZE;
  return apply_run(prec, r, s, work, stream);
}

int pod2g_apply_noalloc(const pod2g_prec *prec, const double *r, double *s, hipStream_t stream) {
  if (!prec || !r || !s) return POD2G_EINVAL;
  if (check_prec(prec)) return POD2G_EINVAL;
  if (pod2g_apply_bytes(prec) > (size_t)POD2G_NOALLOC_SCRATCH_BYTES) return POD2G_ESIZE;
  void *work = nullptr;
  const int st = scratch_address(&work);
  if (st) return st;
  return apply_run(prec, r, s, work, stream);
}

int pod2g_spmv(const pod2g_pattern *pat, const double *vals, int batch, const double *x, double *y,
               hipStream_t stream) {
  if (!pat || !vals || !x || !y || batch < 1 || batch > 65535) return POD2G_EINVAL;
  const int nb = ceil_div(pat->n, NT);
  dim3 grid(nb, batch);
  if (pat->mesh.dim == 2)
    hipLaunchKernelGGL(k_spmv<2>, grid, dim3(NT), 0, stream, pat->n, pat->n_nodes, nb, pat->nvals,
                       pat->colblk, vals, x, y);
  else
    hipLaunchKernelGGL(k_spmv<3>, grid, dim3(NT), 0, stream, pat->n, pat->n_nodes, nb, pat->nvals,
                       pat->colblk, vals, x, y);
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

int pod2g_gauss_seidel(const pod2g_pattern *pat, const double *vals, const double *dinv,
                       int batch, int nsweeps, int backward, const double *b, double *x,
                       hipStream_t stream) {
  if (!pat || !vals || !dinv || !b || !x || batch < 1 || batch > 65535 || nsweeps < 0)
    return POD2G_EINVAL;
  Ctx c;
  memset(&c, 0, sizeof(c));
  c.n = pat->n;
  c.nn = pat->n_nodes;
  c.batch = batch;
  c.nb = ceil_div(pat->n, NT);
  c.nbn = ceil_div(pat->n_nodes, NT);
  c.N = pat->mesh.N;
  c.igroup = 1;
  c.vstride = pat->nvals;
  c.colblk = pat->colblk;
  c.svals = vals;
  c.sdinv = dinv;
  if (pat->mesh.dim == 2) gs_sweeps<2, double>(c, b, x, nsweeps, backward != 0, stream);
  else gs_sweeps<3, double>(c, b, x, nsweeps, backward != 0, stream);
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

int pod2g_jacobi(const pod2g_pattern *pat, const double *vals, const double *dinv, int batch,
                 double omega, int nsweeps, const double *b, double *x, double *tmp,
                 hipStream_t stream) {
  if (!pat || !vals || !dinv || !b || !x || !tmp || batch < 1 || batch > 65535 || nsweeps < 0)
    return POD2G_EINVAL;
  Ctx c;
  memset(&c, 0, sizeof(c));
  c.n = pat->n;
  c.nn = pat->n_nodes;
  c.batch = batch;
  c.nb = ceil_div(pat->n, NT);
  c.nbn = ceil_div(pat->n_nodes, NT);
  c.N = pat->mesh.N;
  c.xwin = choose_xwin(pat);
  c.igroup = default_igroup(batch);
  c.vstride = pat->nvals;
  c.colblk = pat->colblk;
  c.svals = vals;
  c.sdinv = dinv;
  c.omega = omega;
  c.r = const_cast<double *>(b);   // the sweep's right-hand side
  dim3 grid(c.nbn, batch);
  double *cur = x, *oth = tmp;
  for (int i = 0; i < nsweeps; ++i) {
    if (pat->mesh.dim == 2)
      hipLaunchKernelGGL((k_sweep<2, double, false>), grid, dim3(NT), xlds<double>(c), stream, c, cur, oth, 0);
    else
      hipLaunchKernelGGL((k_sweep<3, double, false>), grid, dim3(NT), xlds<double>(c), stream, c, cur, oth, 0);
    double *t = cur; cur = oth; oth = t;
  }
  if (cur != x)
    POD2G_HIP_CHECK(hipMemcpyAsync(x, cur, sizeof(double) * (size_t)pat->n * batch,
                                   hipMemcpyDeviceToDevice, stream));
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

}  // extern "C"
