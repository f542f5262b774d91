// Preconditioner setup: K P, the Galerkin coarse matrix K_c = P^T K P
// (Sec. 2.2 Alg. 2 restrict-and-solve step; Sec. 3.3 Eq. 28), its FP64
// Cholesky factor, FP32 copies for the mixed cycle, and a power-iteration
// estimate of lambda_max(D^-1 K) (damped-Jacobi stability guard).
#include "common.hpp"

#include <math.h>
#include <string.h>

#include <type_traits>

namespace pod2g {

constexpr int KP_CH = 16;  // the node-major basis copy pads k to a multiple of this
constexpr int KC_TR = 64;  // LDS of the coarse-matrix kernel: MAXK x KC_TR doubles twice
constexpr int KC_WG = 256; // workgroups per instance of the coarse-matrix kernel, at most

struct SetupLayout {
  size_t status, lam, pst, arr, kp, L, Linv, kcpart, ppart, p32, d32, kp32, pt, pw, total;
  int nbk;
};

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The FP32 copy of K P pays where a row of K P (k values) is shorter than a
// row of K (27 blocks of 3 in 3D); in 2D (9 blocks of 2) it would not.
static bool want_kp32(int dim, int k, int precision) {
  return precision == POD2G_MIXED && dim == 3 && k > 0;
}

// columns of the node-major basis copy: k rounded up to a multiple of 16,
// zero-padded, so the K P kernel loads whole pieces without bounds tests
static int kp_pad(int k) { return (k + KP_CH - 1) / KP_CH * KP_CH; }

static SetupLayout setup_layout(int n, int k, int batch, int precision, int dim) {
  SetupLayout S;
  // workgroups per instance of the coarse-matrix kernel: at least 8192 rows
  // each, at most KC_WG
  S.nbk = ceil_div(n, 8192);
  if (S.nbk > KC_WG) S.nbk = KC_WG;
  const size_t ntri = (size_t)k * (k + 1) / 2;
  size_t o = 0;
  S.status = o; o += align256(sizeof(int) * batch);
  S.lam = o;    o += align256(sizeof(double) * batch);
  S.pst = o;    o += align256(sizeof(InstState) * batch);
  S.arr = o;    o += sizeof(Arrival) * 2 * (size_t)batch;   // sites: coarse matrix, power step
  S.kp = o;     o += align256(sizeof(double) * (size_t)batch * k * n);
  S.L = o;      o += align256(sizeof(double) * (size_t)batch * k * k);
  S.Linv = o;   o += align256(sizeof(double) * (size_t)batch * k * k);
  S.kcpart = o; o += align256(sizeof(double) * (size_t)batch * S.nbk * (ntri > 0 ? ntri : 1));
  S.ppart = o;  o += align256(sizeof(double) * (size_t)batch * ceil_div(n, NT));
  S.p32 = o;    if (precision == POD2G_MIXED) o += align256(sizeof(float) * (size_t)k * n);
  S.d32 = o;    if (precision == POD2G_MIXED) o += align256(sizeof(float) * (size_t)batch * n);
  S.kp32 = o;   if (want_kp32(dim, k, precision)) o += align256(sizeof(float) * (size_t)batch * k * n);
  S.pt = o;     o += align256(sizeof(double) * (size_t)kp_pad(k) * n);   // node-major copy of P
  S.pw = o;     o += 2 * align256(sizeof(double) * (size_t)batch * n);
  S.total = o;
  return S;
}

__global__ void k_setup_init(InstState *pst, Arrival *arr, int *status, double *lam, int batch,
                             int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  zero_arrivals(arr + (size_t)b * 2, 2, 0, 1);
  InstState s;
  memset(&s, 0, sizeof(s));
  s.xnorm2 = (double)n;
  pst[b] = s;
  status[b] = POD2G_OK;
  lam[b] = 0.0;
}

// Node-major copy of the basis: Pt[node][d][j] = P[j][node dim + d] for
// j < k and 0 up to kpad columns, so that the values K P needs at a
// neighbour node are contiguous per component.
template <int DIM>
__global__ void __launch_bounds__(NT) k_pt(int n, int k, int kpad, const double *__restrict__ P,
                                           double *__restrict__ Pt) {
  const size_t total = (size_t)kpad * n;
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < total; t += (size_t)gridDim.x * NT) {
    const size_t node = t / ((size_t)kpad * DIM);
    const int rem = (int)(t - node * kpad * DIM);
    const int d = rem / kpad, j = rem % kpad;
    Pt[t] = j < k ? P[(size_t)j * n + node * DIM + d] : 0.0;
  }
}

// K P, eight lanes per node (its DIM rows), G instances per thread (grid
// row y holds instances G y .. G y + G - 1): lane q forms columns 16 m + 2 q
// and 16 m + 2 q + 1 for m < M (kpad = 16 M).  The eight lanes of a node
// load the same K values (one request per wave serves them), so K is read
// from memory once for all k columns; for each component of the neighbour
// node the eight lanes read 16 consecutive basis values (128 bytes, one
// 16-byte load each) from the node-major copy Pt, once for the G instances.
// Each entry sums over slots and components in the order of a row-wise
// product.
constexpr int KP_LANES = 8;
typedef double kd2 __attribute__((ext_vector_type(2)));

template <int DIM, int M, int G>
__global__ void __launch_bounds__(NT) k_kp(int n, int nn, int k, int cnt, long long vstride,
                                           const int *__restrict__ colblk,
                                           const double *__restrict__ vals,
                                           const double *__restrict__ Pt, double *__restrict__ KP) {
  const int b0 = blockIdx.y * G;
  const int t = xcd_block(blockIdx.x, gridDim.x) * NT + threadIdx.x;
  const int node = t / KP_LANES, q = t % KP_LANES;
  if (node >= nn) return;
  constexpr int kpad = 16 * M;
  const size_t ns = (size_t)n + DIM;
  const double *vb[G];
#pragma unroll
  for (int g = 0; g < G; ++g) vb[g] = vals + (size_t)min(b0 + g, cnt - 1) * vstride;   // tail: clamped, not stored
  double acc[G][DIM][2 * M];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int r = 0; r < DIM; ++r)
#pragma unroll
      for (int jj = 0; jj < 2 * M; ++jj) acc[g][r][jj] = 0.0;
  auto slot = [&](int s, auto lower) {
    const int c = colblk[s * nn + node];
    const double *pc = Pt + (size_t)c * kpad * DIM + 2 * q;
    kd2 pv[DIM][M];
#pragma unroll
    for (int bc = 0; bc < DIM; ++bc)
#pragma unroll
      for (int m = 0; m < M; ++m) pv[bc][m] = *(const kd2 *)(pc + bc * kpad + 16 * m);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      double kb[DIM][DIM];
      load_block<DIM, double, decltype(lower)::value>(vb[g], s, node, c, nn, ns, kb);
#pragma unroll
      for (int bc = 0; bc < DIM; ++bc)
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
          for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int r = 0; r < DIM; ++r) acc[g][r][2 * m + e] += kb[r][bc] * pv[bc][m][e];
    }
  };
  // lower slots, then the own and upper ones: the order of a row-wise product
  constexpr int H = Half<DIM>::H;
#pragma unroll(G == 1 ? 3 : 1)
  for (int s = 0; s < H; ++s) slot(s, std::true_type());
#pragma unroll(G == 1 ? 3 : 1)
  for (int s = H; s < Stencil<DIM>::S; ++s) slot(s, std::false_type());
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (b0 + g >= cnt) break;
    double *out = KP + (size_t)(b0 + g) * k * n + (size_t)node * DIM;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int j = 16 * m + 2 * q + e;
        if (j < k)
#pragma unroll
          for (int r = 0; r < DIM; ++r) out[(size_t)j * n + r] = acc[g][r][2 * m + e];
      }
  }
}

// G: instances per thread, as many as keep the accumulators (G DIM 2M
// doubles) within about 100 registers
template <int DIM, int M>
static void launch_kp_t(const pod2g_pattern *pat, int cnt, int k, const double *vals,
                        const double *Pt, double *KP, hipStream_t stream) {
  constexpr int G = DIM == 2 ? (M <= 2 ? 4 : 2) : 2;
  dim3 g(ceil_div(pat->n_nodes * KP_LANES, NT), ceil_div(cnt, G));
  hipLaunchKernelGGL((k_kp<DIM, M, G>), g, dim3(NT), 0, stream, pat->n, pat->n_nodes, k, cnt,
                     pat->nvals, pat->colblk, vals, Pt, KP);
}

template <int DIM>
static void launch_kp(const pod2g_pattern *pat, int cnt, int k, const double *vals,
                      const double *Pt, double *KP, hipStream_t stream) {
  switch (kp_pad(k) / 16) {
    case 1: launch_kp_t<DIM, 1>(pat, cnt, k, vals, Pt, KP, stream); break;
    case 2: launch_kp_t<DIM, 2>(pat, cnt, k, vals, Pt, KP, stream); break;
    case 3: launch_kp_t<DIM, 3>(pat, cnt, k, vals, Pt, KP, stream); break;
    default: launch_kp_t<DIM, 4>(pat, cnt, k, vals, Pt, KP, stream); break;
  }
}

__device__ __forceinline__ void tri_index(int e, int &j, int &l) {
  // e = j (j + 1) / 2 + l, 0 <= l <= j
  int jj = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while (jj * (jj + 1) / 2 > e) --jj;
  while ((jj + 1) * (jj + 2) / 2 <= e) ++jj;
  j = jj;
  l = e - jj * (jj + 1) / 2;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Lower triangle of K_c = P^T (K P) on FP64 MFMA (v_mfma_f64_16x16x4f64).
// In step s of a group of four MFMA steps over rows r0 .. r0 + 15, lane
// i + 16 kk holds A[i][kk] = P[j0 + i][r0 + 4 kk + s] and
// B[kk][i] = KP[l0 + i][r0 + 4 kk + s]: a lane's operands of the four steps
// are four consecutive doubles of one row (two 16-byte loads; n is even, so
// each pair lies wholly below or wholly above n).  Every wave accumulates
// the tiles on and below the diagonal over its share of the row groups;
// the workgroup's waves are summed tile by tile in LDS into one partial per
// lower-triangle entry e = j (j + 1) / 2 + l; the last workgroup of an
// instance sums the partials (fixed order) and factors K_c = L L^T in LDS.
// TJ = ceil(k / 16).
template <int TJ>
__global__ void __launch_bounds__(NT) k_kc(int n, int k, int nbk,
                                           const double *__restrict__ P,
                                           const double *__restrict__ KP, double *__restrict__ part,
                                           double *__restrict__ Lout, double *__restrict__ Linv,
                                           int *__restrict__ status, Arrival *arr) {
  __shared__ double sp[MAXK * KC_TR];
  __shared__ double skp[MAXK * KC_TR];
  __shared__ int flag;
  __shared__ int fail;
  constexpr int NTILE = TJ * (TJ + 1) / 2;
  const int b = blockIdx.y, wg = blockIdx.x;
  const int ntri = k * (k + 1) / 2;
  const double *KPb = KP + (size_t)b * k * n;
  const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  const int li = lane & 15, kk = lane >> 4;
  const double *pa[TJ];
  const double *pb[TJ];
#pragma unroll
  for (int t = 0; t < TJ; ++t) {
    const int j = min(t * 16 + li, k - 1);   // rows j >= k: clamped, never used
    pa[t] = P + (size_t)j * n;
    pb[t] = KPb + (size_t)j * n;
  }
  d4 acc[NTILE];
#pragma unroll
  for (int m = 0; m < NTILE; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
  const long long ngroups = (n + 15) / 16, nwaves = (long long)nbk * NWAVE;
  const long long per = (ngroups + nwaves - 1) / nwaves;
  const long long wv = (long long)wg * NWAVE + w;
  const long long gend = min(ngroups, wv * per + per);
  for (long long g0 = wv * per; g0 < gend; ++g0) {
    const int r = (int)(g0 * 16) + 4 * kk;
    const bool ok0 = r < n, ok1 = r + 2 < n;
    d4 a[TJ], c[TJ];
#pragma unroll
    for (int t = 0; t < TJ; ++t) {
      const d2 a0 = *(const d2 *)(pa[t] + (ok0 ? r : 0));
      const d2 a1 = *(const d2 *)(pa[t] + (ok1 ? r + 2 : 0));
      const d2 c0 = *(const d2 *)(pb[t] + (ok0 ? r : 0));
      const d2 c1 = *(const d2 *)(pb[t] + (ok1 ? r + 2 : 0));
      a[t] = d4{ok0 ? a0[0] : 0.0, ok0 ? a0[1] : 0.0, ok1 ? a1[0] : 0.0, ok1 ? a1[1] : 0.0};
      c[t] = d4{c0[0], c0[1], c1[0], c1[1]};
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      int m = 0;
#pragma unroll
      for (int t = 0; t < TJ; ++t)
#pragma unroll
        for (int u = 0; u <= t; ++u, ++m)
          acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t][s4], c[u][s4], acc[m], 0, 0, 0);
    }
  }
  // D[i][jj] of an FP64 tile sits in lane jj + 16 (i % 4), register i / 4
  // (measured; the FP32 16x16x4 layout has lane jj + 16 (i / 4), register i % 4)
  double *buf = sp;   // [NWAVE][16][16]
  double *pw = part + ((size_t)b * nbk + wg) * ntri;
  {
    int m = 0;
#pragma unroll
    for (int t = 0; t < TJ; ++t)
#pragma unroll
      for (int u = 0; u <= t; ++u, ++m) {
#pragma unroll
        for (int v = 0; v < 4; ++v) buf[(w * 16 + kk + 4 * v) * 16 + li] = acc[m][v];
        __syncthreads();
        const int i = threadIdx.x / 16, jj = threadIdx.x % 16;
        const int j = t * 16 + i, l = u * 16 + jj;
        if (j < k && l <= j) {
          double sum = 0.0;
#pragma unroll
          for (int ww = 0; ww < NWAVE; ++ww) sum += buf[(ww * 16 + i) * 16 + jj];
          put_partial(pw + j * (j + 1) / 2 + l, sum);
        }
        __syncthreads();
      }
  }
  double *pbk = part + (size_t)b * nbk * ntri;
  if (!arrive_last(arr + (size_t)b * 2, wg, nbk, &flag)) return;
  // K_c into LDS (full symmetric), then Cholesky
  double *A = sp;  // k x k, row-major
  for (int e = threadIdx.x; e < ntri; e += NT) {
    double s = 0.0;
    for (int ww = 0; ww < nbk; ++ww) s += pbk[(size_t)ww * ntri + e];
    int j, l;
    tri_index(e, j, l);
    A[j * k + l] = s;
    A[l * k + j] = s;
  }
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) {
      const double d = A[j * k + j];
      if (!(d > 0.0)) fail = 1;
      A[j * k + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double d = A[j * k + j];
    for (int i = j + 1 + threadIdx.x; i < k; i += NT) A[i * k + j] /= d;
    __syncthreads();
    const int m = k - j - 1;
    for (int t = threadIdx.x; t < m * m; t += NT) {
      const int i = j + 1 + t / m, l = j + 1 + t % m;
      if (l <= i) A[i * k + l] -= A[i * k + j] * A[l * k + j];
    }
    __syncthreads();
  }
  double *Lb = Lout + (size_t)b * k * k;
  for (int t = threadIdx.x; t < k * k; t += NT) {
    const int i = t / k, l = t % k;
    Lb[t] = l <= i ? A[t] : 0.0;
  }
  // X = L^-1 by forward substitution, one column per thread
  double *X = skp;   // k x k, row-major
  if (threadIdx.x < k) {
    const int j = threadIdx.x;
    for (int i = 0; i < k; ++i) {
      double v = 0.0;
      if (i >= j) {
        v = i == j ? 1.0 : 0.0;
        for (int m = j; m < i; ++m) v -= A[i * k + m] * X[m * k + j];
        v /= A[i * k + i];
      }
      X[i * k + j] = v;
    }
  }
  __syncthreads();
  double *Xb = Linv + (size_t)b * k * k;
  for (int t = threadIdx.x; t < k * k; t += NT) Xb[t] = X[t];
  if (threadIdx.x == 0 && fail) status[b] = POD2G_ENOTSPD;
}

__global__ void __launch_bounds__(NT) k_to_f32(size_t count, const double *__restrict__ a,
                                               float *__restrict__ o) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT)
    o[i] = (float)a[i];
}

__global__ void __launch_bounds__(NT) k_fill(size_t count, double v, double *__restrict__ o) {
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT)
    o[i] = v;
}

// y = D^-1 K x / ||x||, ||y||^2; last block: lambda estimate = ||y||.
template <int DIM>
__global__ void __launch_bounds__(NT) k_power(int n, int nn, int nb, long long vstride,
                                              const int *__restrict__ colblk,
                                              const double *__restrict__ vals,
                                              const double *__restrict__ dinv,
                                              const double *__restrict__ x, double *__restrict__ y,
                                              double *__restrict__ part, InstState *pst, Arrival *arr,
                                              double *lam) {
  __shared__ double lds[NWAVE];
  __shared__ int flag;
  const int b = blockIdx.y;
  const int blk = xcd_block(blockIdx.x, nb);
  const int row = blk * NT + threadIdx.x;
  const size_t off = (size_t)b * n;
  const double inv = 1.0 / sqrt(pst[b].xnorm2);
  double yy = 0.0;
  if (row < n) {
    const double kx = row_dot<DIM>(colblk, vals + (size_t)b * vstride, x + off, row, row / DIM, n, nn);
    const double v = dinv[off + row] * kx * inv;
    y[off + row] = v;
    yy = v * v;
  }
  yy = block_sum(yy, lds);
  if (threadIdx.x == 0) put_partial(part + (size_t)b * nb + blk, yy);
  if (!arrive_last(arr + (size_t)b * 2 + 1, blk, nb, &flag)) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s += part[(size_t)b * nb + i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) {
    pst[b].xnorm2 = s;
    lam[b] = sqrt(s);
  }
}

__global__ void k_smoother_guard(int batch, double omega, const double *lam, int *status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  if (status[b] == POD2G_OK && !(omega * lam[b] < 2.0)) status[b] = POD2G_ESMOOTHER;
}

}  // namespace pod2g

using namespace pod2g;

extern "C" {

size_t pod2g_setup_bytes(const pod2g_pattern *pat, int k, int batch, int precision) {
  if (!pat || k < 0 || k > MAXK || batch < 1) return 0;
  return setup_layout(pat->n, k, batch, precision, pat->mesh.dim).total;
}

}  // extern "C"

// Setup kernels for instances b0 .. b0 + cnt - 1 of handle pr, whose
// buffers sit in the setup workspace w with layout S (for pr.batch).
static int setup_run(const pod2g_prec &pr, const SetupLayout &S, char *w, int b0, int cnt,
                     int power_iters, bool convert_p, hipStream_t stream) {
  const pod2g_pattern *pat = &pr.pat;
  const int n = pat->n, dim = pat->mesh.dim, k = pr.k;
  const size_t ntri = (size_t)k * (k + 1) / 2;
  const int nb = ceil_div(n, NT);
  const double *vals = pr.vals + (size_t)b0 * pat->nvals;
  const double *dinv = pr.dinv + (size_t)b0 * n;
  int *status = pr.status + b0;
  double *lam = pr.lam + b0;
  InstState *pst = (InstState *)(w + S.pst) + b0;
  Arrival *arr = (Arrival *)(w + S.arr) + (size_t)b0 * 2;
  double *KP = k > 0 ? pr.KP + (size_t)b0 * k * n : nullptr;
  double *L = k > 0 ? pr.L + (size_t)b0 * k * k : nullptr;
  double *Linv = k > 0 ? pr.Linv + (size_t)b0 * k * k : nullptr;
  double *kcpart = (double *)(w + S.kcpart) + (size_t)b0 * S.nbk * (ntri > 0 ? ntri : 1);
  double *ppart = (double *)(w + S.ppart) + (size_t)b0 * nb;
  double *pw0 = (double *)(w + S.pw) + (size_t)b0 * n;
  double *pw1 = (double *)(w + S.pw + align256(sizeof(double) * (size_t)pr.batch * n)) + (size_t)b0 * n;

  hipLaunchKernelGGL(k_setup_init, dim3(ceil_div(cnt, 64)), dim3(64), 0, stream, pst, arr, status, lam,
                     cnt, n);
  if (k > 0) {
    double *Pt = (double *)(w + S.pt);
    if (convert_p) {
      if (dim == 2)
        hipLaunchKernelGGL(k_pt<2>, dim3(2048), dim3(NT), 0, stream, n, k, kp_pad(k), pr.P, Pt);
      else
        hipLaunchKernelGGL(k_pt<3>, dim3(2048), dim3(NT), 0, stream, n, k, kp_pad(k), pr.P, Pt);
    }
    if (dim == 2) launch_kp<2>(pat, cnt, k, vals, (const double *)Pt, KP, stream);
    else launch_kp<3>(pat, cnt, k, vals, (const double *)Pt, KP, stream);
    {
      const dim3 gc(S.nbk, cnt);
      const double *kpc = KP;
      switch ((k + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_kc<1>, gc, dim3(NT), 0, stream, n, k, S.nbk, pr.P, kpc, kcpart, L, Linv, status, arr); break;
        case 2: hipLaunchKernelGGL(k_kc<2>, gc, dim3(NT), 0, stream, n, k, S.nbk, pr.P, kpc, kcpart, L, Linv, status, arr); break;
        case 3: hipLaunchKernelGGL(k_kc<3>, gc, dim3(NT), 0, stream, n, k, S.nbk, pr.P, kpc, kcpart, L, Linv, status, arr); break;
        default: hipLaunchKernelGGL(k_kc<4>, gc, dim3(NT), 0, stream, n, k, S.nbk, pr.P, kpc, kcpart, L, Linv, status, arr); break;
      }
    }
    if (convert_p && pr.precision == POD2G_MIXED)
      hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(NT), 0, stream, (size_t)k * n, pr.P, pr.P32);
    if (pr.KP32)
      hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(NT), 0, stream, (size_t)cnt * k * n,
                         (const double *)KP, pr.KP32 + (size_t)b0 * k * n);
  }
  if (pr.precision == POD2G_MIXED)
    hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(NT), 0, stream, (size_t)cnt * n, dinv,
                       pr.dinv32 + (size_t)b0 * n);
  if (power_iters > 0) {
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(NT), 0, stream, (size_t)cnt * n, 1.0, pw0);
    double *x = pw0, *y = pw1;
    for (int it = 0; it < power_iters; ++it) {
      if (dim == 2)
        hipLaunchKernelGGL(k_power<2>, dim3(nb, cnt), dim3(NT), 0, stream, n, pat->n_nodes, nb,
                           pat->nvals, pat->colblk, vals, dinv, (const double *)x, y, ppart, pst, arr, lam);
      else
        hipLaunchKernelGGL(k_power<3>, dim3(nb, cnt), dim3(NT), 0, stream, n, pat->n_nodes, nb,
                           pat->nvals, pat->colblk, vals, dinv, (const double *)x, y, ppart, pst, arr, lam);
      double *t = x; x = y; y = t;
    }
    hipLaunchKernelGGL(k_smoother_guard, dim3(ceil_div(cnt, 64)), dim3(64), 0, stream, cnt,
                       pr.omega, (const double *)lam, status);
  }
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

extern "C" {

int pod2g_setup(const pod2g_pattern *pat, const double *vals, const float *vals32,
                const double *dinv, const double *P, int k, double omega, int nu_pre, int nu_post,
                int precision, int batch, int power_iters, void *work, size_t bytes,
                pod2g_prec *out, hipStream_t stream) {
  if (!pat || !vals || !dinv || !work || !out) return POD2G_EINVAL;
  if (k < 0 || k > MAXK || (k > 0 && !P) || batch < 1 || batch > 65535) return POD2G_EINVAL;
  if (k > 0 && ((uintptr_t)P & 15)) return POD2G_EINVAL;   // read in 16-byte pieces
  if (precision != POD2G_FP64 && precision != POD2G_MIXED) return POD2G_EINVAL;
  if (precision == POD2G_MIXED && !vals32) return POD2G_EINVAL;
  if (!(omega > 0.0) || nu_pre < 0 || nu_post < 0 || nu_pre > 64 || nu_post > 64 || power_iters < 0)
    return POD2G_EINVAL;
  if (bytes < pod2g_setup_bytes(pat, k, batch, precision)) return POD2G_ESIZE;
  const int n = pat->n;
  SetupLayout S = setup_layout(n, k, batch, precision, pat->mesh.dim);
  char *w = (char *)work;
  pod2g_prec pr;
  memset(&pr, 0, sizeof(pr));
  pr.pat = *pat;
  pr.batch = batch;
  pr.k = k;
  pr.nu_pre = nu_pre;
  pr.nu_post = nu_post;
  pr.precision = precision;
  pr.omega = omega;
  pr.vals = vals;
  pr.vals32 = precision == POD2G_MIXED ? vals32 : nullptr;
  pr.dinv = dinv;
  pr.P = P;
  pr.status = (int *)(w + S.status);
  pr.lam = (double *)(w + S.lam);
  pr.KP = k > 0 ? (double *)(w + S.kp) : nullptr;
  pr.L = k > 0 ? (double *)(w + S.L) : nullptr;
  pr.Linv = k > 0 ? (double *)(w + S.Linv) : nullptr;
  pr.P32 = (precision == POD2G_MIXED && k > 0) ? (float *)(w + S.p32) : nullptr;
  pr.dinv32 = precision == POD2G_MIXED ? (float *)(w + S.d32) : nullptr;
  pr.KP32 = want_kp32(pat->mesh.dim, k, precision) ? (float *)(w + S.kp32) : nullptr;
  pr.work = work;
  pr.smoother = POD2G_SMOOTHER_JACOBI;
  int st = setup_run(pr, S, w, 0, batch, power_iters, true, stream);
  if (st) return st;
  *out = pr;
  return POD2G_OK;
}

int pod2g_set_smoother(pod2g_prec *prec, int smoother) {
  if (!prec || (smoother != POD2G_SMOOTHER_JACOBI && smoother != POD2G_SMOOTHER_SGS))
    return POD2G_EINVAL;
  prec->smoother = smoother;
  return POD2G_OK;
}

int pod2g_setup_slot(const pod2g_prec *prec, int slot, int power_iters, hipStream_t stream) {
  if (!prec || !prec->work || !prec->status || slot < 0 || slot >= prec->batch || power_iters < 0)
    return POD2G_EINVAL;
  if (prec->k < 0 || prec->k > MAXK || (prec->k > 0 && (!prec->P || !prec->KP)) ||
      (prec->precision == POD2G_MIXED && !prec->dinv32))
    return POD2G_EINVAL;
  SetupLayout S = setup_layout(prec->pat.n, prec->k, prec->batch, prec->precision,
                                 prec->pat.mesh.dim);
  return setup_run(*prec, S, (char *)prec->work, slot, 1, power_iters, false, stream);
}

int pod2g_setup_status(const pod2g_prec *prec, int *status_h, double *lam_h, hipStream_t stream) {
  if (!prec || !status_h || !prec->status) return POD2G_EINVAL;
  POD2G_HIP_CHECK(hipMemcpyAsync(status_h, prec->status, sizeof(int) * prec->batch,
                                 hipMemcpyDeviceToHost, stream));
  if (lam_h)
    POD2G_HIP_CHECK(hipMemcpyAsync(lam_h, prec->lam, sizeof(double) * prec->batch,
                                   hipMemcpyDeviceToHost, stream));
  POD2G_HIP_CHECK(hipStreamSynchronize(stream));
  return POD2G_OK;
}

}  // extern "C"
