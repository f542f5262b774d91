// Shared device helpers of the POD-2G library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pod2g.h"

namespace pod2g {

constexpr int NT = 256;          // threads per workgroup of the row kernels
constexpr int WAVE = 64;
constexpr int NWAVE = NT / WAVE;
constexpr int MAXK = POD2G_MAX_K;

// Per-instance solver state (one cache line pair, device memory).
struct alignas(128) InstState {
  double rho;      // r^T s of the current iterate
  double gamma;    // p^T K p
  double alpha, beta;
  double rr;       // ||r||^2 (recursive residual)
  double ff;       // ||f||^2
  double tol2;     // (rtol ||f||)^2
  double rs_prev;  // r_{k+1}^T s_k (flexible beta)
  double rr_true;  // ||f - K u||^2 at the last true-residual check
  double xnorm2;   // power iteration: ||x||^2
  double scale;    // power-of-two scale of the FP32 cycle input
  double pad0;
  int iter, maxit, done, status;
  int restart;     // next beta is forced to 0
  int beta_kind;
  int checked;     // served solve: the true residual of the final iterate is known
  int pending;     // served solve: r is replaced by the true residual in the next update
  int fresh;       // served solve: admitted, r0 = f - K x0 not formed yet
  int pad1;
};

// Reduction sites of one instance; each has its own arrival counters.
enum CounterSlot { CNT_A = 0, CNT_B = 1, CNT_C = 2, CNT_D = 3, CNT_E = 4, CNT_F = 5, NSITE = 8 };

// Arrival counters of one reduction site: a workgroup counts on the counter
// of its group (block index mod ARR_GROUPS), the last of each group on the
// top counter.  Atomics on one address serialise (about 12 ns each), so a
// single counter for hundreds of workgroups puts microseconds on the
// critical path of every reduction; two levels of at most ~32 arrivals
// keep that chain short.  Each counter has its own 128-byte line.
constexpr int ARR_GROUPS = 32;
struct alignas(128) ArrCounter {
  unsigned v;
  unsigned pad[31];
};
struct Arrival {
  ArrCounter top;
  ArrCounter grp[ARR_GROUPS];
};

// Zero the counters of `count` sites (one thread per site and counter).
__device__ __forceinline__ void zero_arrivals(Arrival *a, int count, int tid, int nthreads) {
  for (int i = tid; i < count * (ARR_GROUPS + 1); i += nthreads) {
    Arrival *s = a + i / (ARR_GROUPS + 1);
    const int j = i % (ARR_GROUPS + 1);
    if (j == 0) s->top.v = 0u;
    else s->grp[j - 1].v = 0u;
  }
}

// Blocks are handed to the 8 XCDs round-robin; map them so that every XCD
// works on one contiguous range of rows (its L2 then holds that range's
// neighbourhood of the gathered vector).  A bijection for any nblocks.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int q = nblocks >> 3, rem = nblocks & 7;
  const int x = bid & 7, idx = bid >> 3;
  return x * q + (x < rem ? x : rem) + idx;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum over the workgroup in a fixed order; result valid on thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds /*[NWAVE]*/) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) t += lds[i];
  }
  __syncthreads();
  return t;
}

// Two sums at once (one pass of barriers).
__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds /*[2*NWAVE]*/) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) { lds[w] = a; lds[NWAVE + w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int i = 0; i < NWAVE; ++i) { ta += lds[i]; tb += lds[NWAVE + i]; }
    a = ta; b = tb;
  }
  __syncthreads();
}

// Cross-workgroup partial results: each workgroup writes its partials with
// agent-scope relaxed atomic stores, which write through to the point of
// coherence shared by all XCDs (no L2 writeback of unrelated data).  The
// last workgroup to arrive invalidates its caches once (agent-scope acquire
// fence) and then reads the partials with ordinary, pipelined loads.
__device__ __forceinline__ void put_partial(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Report whether this workgroup (block index blk of `total`) is the last to
// arrive at the site.  Every wave first waits for its outstanding stores
// (so its put_partial writes are complete before the counters move); the
// last workgroup of a group resets the group counter, the last of all the
// top counter; it then acquires and may read every partial.
__device__ __forceinline__ bool arrive_last(Arrival *a, int blk, unsigned total, int *lds_flag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = (unsigned)blk % ARR_GROUPS;
    const unsigned members = total / ARR_GROUPS + (g < total % ARR_GROUPS ? 1u : 0u);
    int last = 0;
    const unsigned prev = __hip_atomic_fetch_add(&a->grp[g].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == members - 1u) {
      __hip_atomic_store(&a->grp[g].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned groups = total < (unsigned)ARR_GROUPS ? total : (unsigned)ARR_GROUPS;
      const unsigned p2 = __hip_atomic_fetch_add(&a->top.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = (p2 == groups - 1u);
      if (last) __hip_atomic_store(&a->top.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    *lds_flag = last;
  }
  __syncthreads();
  const bool last = *lds_flag != 0;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// Deterministic sum of m partials (strided by `stride` doubles) by one
// workgroup: fixed per-thread order, then the fixed block tree.
// Sum of part[i * stride] for i = first, first + step, ... < m with eight
// independent accumulators: the partials come from other XCDs (a trip to
// the memory side each), so up to eight loads per thread are in flight
// together.  The order is fixed by m and step.
__device__ __forceinline__ double strided_sum(const double *part, int first, int m, int step,
                                              int stride) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (m <= 0) return 0.0;
  int i = first;
  for (; i + 7 * step < m; i += 8 * step) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += part[(size_t)(i + u * step) * stride];
  }
  // the remainder: indices clamped into range so that no load is guarded
  // (a guarded load is a branch, and the compiler then waits for each
  // before the next), the surplus discarded afterwards
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int iu = i + u * step;
    v[u] = part[(size_t)(iu < m ? iu : m - 1) * stride];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (i + u * step < m) a[u] += v[u];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// As strided_sum, but all loads of a share of up to WIDE partials are
// issued before any is added (one trip to the memory side per WIDE
// partials instead of per eight), then summed by a fixed pairwise tree.
constexpr int WIDE = 48;
__device__ __forceinline__ double strided_sum_wide(const double *part, int first, int m, int step,
                                                   int stride) {
  double total = 0.0;
  for (int base = first; base < m; base += WIDE * step) {
    double v[WIDE];
    // unguarded loads (clamped into range, zeroed afterwards), all in flight
#pragma unroll
    for (int u = 0; u < WIDE; ++u) {
      const int i = base + u * step;
      v[u] = part[(size_t)(i < m ? i : m - 1) * stride];
    }
#pragma unroll
    for (int u = 0; u < WIDE; ++u)
      if (base + u * step >= m) v[u] = 0.0;
#pragma unroll
    for (int w = 1; w < WIDE; w <<= 1)
#pragma unroll
      for (int u = 0; u + w < WIDE; u += 2 * w) v[u] += v[u + w];
    total += v[0];
  }
  return total;
}

__device__ __forceinline__ double reduce_partials(const double *part, int m, int stride,
                                                  double *lds) {
  return block_sum(strided_sum(part, threadIdx.x, m, NT, stride), lds);
}

__device__ __forceinline__ bool finite(double x) { return x - x == 0.0; }

template <int DIM> struct Stencil {
  static constexpr int S = DIM == 2 ? 9 : 27;   // block slots per node
  static constexpr int NE = DIM == 2 ? 4 : 8;   // nodes per element
  static constexpr int ED = DIM * NE;           // element DOFs
};

// Symmetric (half) block-ELL storage.  K is symmetric, so only the centre
// slot and the "upper" slots of every node are stored -- slot s >= H = S/2,
// i.e. neighbour offset (dz, dy, dx) > 0 in that order -- with a zero node
// after the last node of every plane:
//   vals[((s - H) DIM + b) ns + node DIM + r] = K(node DIM + r, nb_s(node) DIM + b),
//   ns = n + DIM (plane stride).
// A lower slot s < H of node i is the transpose of the upper slot S - 1 - s
// of its neighbour j = nb_s(i): K(i DIM + r, j DIM + b) =
// vals[((H - s) DIM + r) ns + j DIM + b].  An absent neighbour (colblk
// points at the node itself) reads the zero node instead.  The values are
// the same numbers full storage would hold (assembly is exactly symmetric),
// so every product sums the same terms in the same order.
template <int DIM> struct Half {
  static constexpr int S = Stencil<DIM>::S;
  static constexpr int H = S / 2;        // the centre slot
  static constexpr int SH = H + 1;       // stored slots per node
};

// The DIM x DIM block K(node, nb_s(node)) as m[r][b]; c = colblk[s][node].
// LOWER: s < H (read transposed at the neighbour), else s >= H; a compile-
// time choice, so that callers iterate over the lower and the upper slots in
// two loops and no load sits behind a run-time branch (the compiler would
// then wait for it before going on).
template <int DIM, typename T, bool LOWER>
__device__ __forceinline__ void load_block(const T *__restrict__ vals, int s, int node, int c,
                                           int nn, size_t ns, T m[DIM][DIM]) {
  constexpr int H = Half<DIM>::H;
  if (!LOWER) {
    const T *v = vals + (size_t)((s - H) * DIM) * ns + (size_t)node * DIM;
#pragma unroll
    for (int b = 0; b < DIM; ++b)
#pragma unroll
      for (int r = 0; r < DIM; ++r) m[r][b] = v[(size_t)b * ns + r];
  } else {
    const int j = c == node ? nn : c;
    const T *v = vals + (size_t)((H - s) * DIM) * ns + (size_t)j * DIM;
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
      for (int b = 0; b < DIM; ++b) m[r][b] = v[(size_t)r * ns + b];
  }
}

// (K x)_row; x is gathered at the neighbour DOFs.  Lower slots, then upper
// ones: the same order s = 0 .. S - 1 as a row-wise product.
template <int DIM, typename T, typename XT>
__device__ __forceinline__ T row_dot(const int *__restrict__ colblk, const T *__restrict__ vals,
                                     const XT *__restrict__ x, int row, int node, int n, int nn) {
  constexpr int S = Stencil<DIM>::S, H = Half<DIM>::H;
  const size_t ns = (size_t)n + DIM;
  const int r = row - node * DIM;
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < H; ++s) {
    const int c = colblk[s * nn + node];
    const int j = c == node ? nn : c;
    const T *v = vals + (size_t)((H - s) * DIM + r) * ns + (size_t)j * DIM;
#pragma unroll
    for (int b = 0; b < DIM; ++b) acc += v[b] * (T)x[c * DIM + b];
  }
#pragma unroll
  for (int s = H; s < S; ++s) {
    const int c = colblk[s * nn + node];
    const T *v = vals + (size_t)((s - H) * DIM) * ns + row;
#pragma unroll
    for (int b = 0; b < DIM; ++b) acc += v[(size_t)b * ns] * (T)x[c * DIM + b];
  }
  return acc;
}

// One slot's contribution to (K x) of the node's DIM rows.
template <int DIM, typename T, bool LOWER, typename XG>
__device__ __forceinline__ void node_slot(const int *__restrict__ colblk, const T *__restrict__ vals,
                                          XG xg, int s, int node, int nn, size_t ns, T acc[DIM]) {
  const int c = colblk[s * nn + node];
  T xv[DIM];
#pragma unroll
  for (int b = 0; b < DIM; ++b) xv[b] = (T)xg((size_t)c * DIM + b);
  T m[DIM][DIM];
  load_block<DIM, T, LOWER>(vals, s, node, c, nn, ns, m);
#pragma unroll
  for (int b = 0; b < DIM; ++b)
#pragma unroll
    for (int r = 0; r < DIM; ++r) acc[r] += m[r][b] * xv[b];
}

// (K x) for the DIM rows of one node (row = node DIM + r): per neighbour
// slot one index load, one DIM-wide gather xg(c DIM + b) and the block's
// DIM x DIM values (the node's rows are adjacent in every stored plane; a
// lower block's rows are adjacent at the neighbour).  Each row sums in the
// order of row_dot, so the results agree with it bit for bit.  UNR: slots
// unrolled together; 0 = all (every slot's loads in flight at once), a
// smaller count for gathers that compute their value from several vectors
// (all 27 slots of those need more than 256 registers).
template <int DIM, typename T, typename XG, int UNR = 0>
__device__ __forceinline__ void node_dot(const int *__restrict__ colblk, const T *__restrict__ vals,
                                         XG xg, int node, int n, int nn, T acc[DIM]) {
  constexpr int S = Stencil<DIM>::S, H = Half<DIM>::H;
  const size_t ns = (size_t)n + DIM;
#pragma unroll
  for (int r = 0; r < DIM; ++r) acc[r] = T(0);
#pragma unroll(UNR > 0 ? UNR : H)
  for (int s = 0; s < H; ++s) node_slot<DIM, T, true>(colblk, vals, xg, s, node, nn, ns, acc);
#pragma unroll(UNR > 0 ? UNR : S - H)
  for (int s = H; s < S; ++s) node_slot<DIM, T, false>(colblk, vals, xg, s, node, nn, ns, acc);
}

inline int ceil_div(long long a, int b) { return (int)((a + b - 1) / b); }

}  // namespace pod2g

#define POD2G_HIP_CHECK(expr)                  \
  do {                                         \
    if ((expr) != hipSuccess) return POD2G_EHIP; \
  } while (0)
