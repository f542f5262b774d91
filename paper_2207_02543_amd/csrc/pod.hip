// Offline POD by the method of snapshots (Sec. 3.3, steps 1-2):
// G = U^T U, its eigenpairs by cyclic Jacobi rotations, and
// P = U Psi_k Lambda_k^{-1/2} (Eq. 26) for the k largest eigenvalues.
#include "common.hpp"

#include <math.h>
#include <string.h>
#include <vector>

namespace pod2g {

constexpr int GT = 32;        // Gram output tile (GT x GT entries per workgroup)
constexpr int GR = 64;        // snapshot rows per LDS stage
constexpr int MAXN = 256;     // largest snapshot count
constexpr int EIG_NT = 1024;  // threads of the eigensolver workgroup
constexpr int BAS_CH = 16;    // basis columns per pass over U

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct PodLayout {
  size_t gpart, G, V, W, lamh, total;
  int chunks;
};

static PodLayout pod_layout(int n, int N, int k) {
  PodLayout L;
  int chunks = n / (GR * 64);
  if (chunks < 1) chunks = 1;
  if (chunks > 256) chunks = 256;
  L.chunks = chunks;
  size_t o = 0;
  L.gpart = o; o += align256(sizeof(double) * (size_t)chunks * N * N);
  L.G = o;     o += align256(sizeof(double) * (size_t)N * N);
  L.V = o;     o += align256(sizeof(double) * (size_t)N * N);
  L.W = o;     o += align256(sizeof(double) * (size_t)N * (k > 0 ? k : 1));
  L.lamh = o;  o += align256(sizeof(double) * (size_t)N);
  L.total = o;
  return L;
}

// Partial Gram tile (ti, tj) over the rows of chunk blockIdx.z: one thread
// per 4 entries of the 32 x 32 tile.  Tiles above the diagonal are skipped.
__global__ void __launch_bounds__(NT) k_gram(int n, int N, int chunks, const double *__restrict__ U,
                                             double *__restrict__ part) {
  const int ti = blockIdx.x, tj = blockIdx.y, ch = blockIdx.z;
  if (tj > ti) return;
  __shared__ double a[GT * GR], b[GT * GR];
  const long long per = ((long long)n + chunks - 1) / chunks;
  const long long r_begin = per * ch;
  const long long r_end = r_begin + per < n ? r_begin + per : n;
  const int i0 = ti * GT, j0 = tj * GT;
  double acc[4] = {0, 0, 0, 0};
  const int li = threadIdx.x / 8;         // 0..31 tile row
  const int lj = (threadIdx.x % 8) * 4;   // 4 consecutive tile columns
  for (long long r0 = r_begin; r0 < r_end; r0 += GR) {
    for (int t = threadIdx.x; t < GT * GR; t += NT) {
      const int c = t / GR, rr = t % GR;
      const long long row = r0 + rr;
      const bool ok = row < r_end;
      a[t] = (ok && i0 + c < N) ? U[(size_t)(i0 + c) * n + row] : 0.0;
      b[t] = (ok && j0 + c < N) ? U[(size_t)(j0 + c) * n + row] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < GR; ++rr) {
      const double av = a[li * GR + rr];
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] += av * b[(lj + m) * GR + rr];
    }
    __syncthreads();
  }
  double *pc = part + (size_t)ch * N * N;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = i0 + li, j = j0 + lj + m;
    if (i < N && j < N && j <= i) pc[(size_t)i * N + j] = acc[m];
  }
}

// G = sum over chunks (fixed order), mirrored to the upper triangle.
__global__ void __launch_bounds__(NT) k_gram_reduce(int N, int chunks, const double *__restrict__ part,
                                                    double *__restrict__ G) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= N * N) return;
  const int i = e / N, j = e % N;
  if (j > i) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[(size_t)c * N * N + e];
  G[(size_t)i * N + j] = s;
  G[(size_t)j * N + i] = s;
}

// Cyclic Jacobi eigensolver for the symmetric N x N matrix G (in place;
// eigenvalues end on the diagonal), eigenvectors accumulated in V.  Rounds
// of N/2 disjoint rotations (circle-method pairing) run in parallel; each
// rotation J (J_pp = J_qq = c, J_pq = s, J_qp = -s) annihilates G_pq in
// G <- J^T G J.  Single workgroup.
__global__ void __launch_bounds__(EIG_NT) k_jacobi_eig(int N, double *__restrict__ G,
                                                       double *__restrict__ V, int max_sweeps) {
  __shared__ int pp[MAXN / 2], pq[MAXN / 2];
  __shared__ double cs[MAXN / 2], sn[MAXN / 2];
  __shared__ double red[EIG_NT / WAVE];
  __shared__ int stop;
  const int Np = N + (N & 1);
  const int half = Np / 2;
  for (int t = threadIdx.x; t < N * N; t += EIG_NT) V[t] = (t / N == t % N) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // off-diagonal and total Frobenius mass
    double off = 0.0, tot = 0.0;
    for (int t = threadIdx.x; t < N * N; t += EIG_NT) {
      const double g = G[t];
      tot += g * g;
      if (t / N != t % N) off += g * g;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = off;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < EIG_NT / WAVE; ++i) s += red[i];
      off = s;
    }
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < EIG_NT / WAVE; ++i) s += red[i];
      stop = !(off > 1e-32 * s);
    }
    __syncthreads();
    if (stop) break;
    for (int round = 0; round < Np - 1; ++round) {
      for (int t = threadIdx.x; t < half; t += EIG_NT) {
        const int pa = t, pb = Np - 1 - t;
        const int p = pa == 0 ? 0 : 1 + (pa - 1 + round) % (Np - 1);
        const int q = pb == 0 ? 0 : 1 + (pb - 1 + round) % (Np - 1);
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        double c = 1.0, s = 0.0;
        if (hi < N) {
          const double apq = G[(size_t)lo * N + hi];
          if (apq != 0.0) {
            const double app = G[(size_t)lo * N + lo], aqq = G[(size_t)hi * N + hi];
            const double theta = (aqq - app) / (2.0 * apq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
          }
        }
        pp[t] = lo;
        pq[t] = hi;
        cs[t] = c;
        sn[t] = s;
      }
      __syncthreads();
      // columns: G J and V J
      for (int t = threadIdx.x; t < half * N; t += EIG_NT) {
        const int pr = t / N, i = t % N;
        const int p = pp[pr], q = pq[pr];
        if (q >= N || sn[pr] == 0.0) continue;
        const double c = cs[pr], s = sn[pr];
        const double gp = G[(size_t)i * N + p], gq = G[(size_t)i * N + q];
        G[(size_t)i * N + p] = c * gp - s * gq;
        G[(size_t)i * N + q] = s * gp + c * gq;
        const double vp = V[(size_t)i * N + p], vq = V[(size_t)i * N + q];
        V[(size_t)i * N + p] = c * vp - s * vq;
        V[(size_t)i * N + q] = s * vp + c * vq;
      }
      __syncthreads();
      // rows: J^T (G J)
      for (int t = threadIdx.x; t < half * N; t += EIG_NT) {
        const int pr = t / N, i = t % N;
        const int p = pp[pr], q = pq[pr];
        if (q >= N || sn[pr] == 0.0) continue;
        const double c = cs[pr], s = sn[pr];
        const double gp = G[(size_t)p * N + i], gq = G[(size_t)q * N + i];
        G[(size_t)p * N + i] = c * gp - s * gq;
        G[(size_t)q * N + i] = s * gp + c * gq;
      }
      __syncthreads();
      // the rotated pair's off-diagonal entries are zero in exact arithmetic
      for (int t = threadIdx.x; t < half; t += EIG_NT) {
        const int p = pp[t], q = pq[t];
        if (q < N && sn[t] != 0.0) {
          G[(size_t)p * N + q] = 0.0;
          G[(size_t)q * N + p] = 0.0;
        }
      }
      __syncthreads();
    }
  }
}

// Sort eigenvalues descending; W[:, j] = V[:, idx_j] / sqrt(lambda_j).
__global__ void k_eig_sort(int N, int k, const double *__restrict__ G, const double *__restrict__ V,
                           double *__restrict__ lam, double *__restrict__ W) {
  __shared__ int order[MAXN];
  __shared__ double ev[MAXN];
  for (int i = threadIdx.x; i < N; i += blockDim.x) ev[i] = G[(size_t)i * N + i];
  __syncthreads();
  if (threadIdx.x == 0) {
    // stable insertion sort by value, descending (N <= 256)
    for (int i = 0; i < N; ++i) order[i] = i;
    for (int i = 1; i < N; ++i) {
      const int key = order[i];
      int j = i - 1;
      while (j >= 0 && ev[order[j]] < ev[key]) { order[j + 1] = order[j]; --j; }
      order[j + 1] = key;
    }
    for (int i = 0; i < N; ++i) lam[i] = ev[order[i]];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N * k; t += blockDim.x) {
    const int i = t / k, j = t % k;
    const double l = ev[order[j]];
    W[(size_t)i * k + j] = l > 0.0 ? V[(size_t)i * N + order[j]] / sqrt(l) : 0.0;
  }
}

// P[:, j0 ..] = U W[:, j0 ..]: one thread per row, BAS_CH columns per pass.
__global__ void __launch_bounds__(NT) k_basis(int n, int N, int k, const double *__restrict__ U,
                                              const double *__restrict__ W, double *__restrict__ P) {
  __shared__ double w[MAXN * BAS_CH];
  const int j0 = blockIdx.y * BAS_CH;
  const int jn = k - j0 < BAS_CH ? k - j0 : BAS_CH;
  for (int t = threadIdx.x; t < N * BAS_CH; t += NT) {
    const int i = t / BAS_CH, jj = t % BAS_CH;
    w[t] = jj < jn ? W[(size_t)i * k + j0 + jj] : 0.0;
  }
  __syncthreads();
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  double acc[BAS_CH];
#pragma unroll
  for (int jj = 0; jj < BAS_CH; ++jj) acc[jj] = 0.0;
  for (int i = 0; i < N; ++i) {
    const double u = U[(size_t)i * n + row];
#pragma unroll
    for (int jj = 0; jj < BAS_CH; ++jj) acc[jj] += u * w[i * BAS_CH + jj];
  }
#pragma unroll
  for (int jj = 0; jj < BAS_CH; ++jj)
    if (jj < jn) P[(size_t)(j0 + jj) * n + row] = acc[jj];
}

}  // namespace pod2g

using namespace pod2g;

extern "C" {

size_t pod2g_pod_basis_bytes(int n, int N, int k) {
  if (n < 1 || N < 1 || N > MAXN || k < 1 || k > MAXK || k > N) return 0;
  return pod_layout(n, N, k).total;
}

int pod2g_pod_basis(const double *U, int n, int N, int k, double *P, double *lam, void *work,
                    size_t bytes, hipStream_t stream) {
  if (!U || !P || !lam || !work) return POD2G_EINVAL;
  if (n < 1 || N < 1 || N > MAXN || k < 1 || k > MAXK || k > N) return POD2G_EINVAL;
  if (bytes < pod2g_pod_basis_bytes(n, N, k)) return POD2G_ESIZE;
  PodLayout L = pod_layout(n, N, k);
  char *w = (char *)work;
  double *gpart = (double *)(w + L.gpart), *G = (double *)(w + L.G), *V = (double *)(w + L.V);
  double *W = (double *)(w + L.W);
  const int tiles = ceil_div(N, GT);
  hipLaunchKernelGGL(k_gram, dim3(tiles, tiles, L.chunks), dim3(NT), 0, stream, n, N, L.chunks, U, gpart);
  hipLaunchKernelGGL(k_gram_reduce, dim3(ceil_div((long long)N * N, NT)), dim3(NT), 0, stream, N,
                     L.chunks, (const double *)gpart, G);
  hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(EIG_NT), 0, stream, N, G, V, 60);
  hipLaunchKernelGGL(k_eig_sort, dim3(1), dim3(NT), 0, stream, N, k, (const double *)G,
                     (const double *)V, lam, W);
  hipLaunchKernelGGL(k_basis, dim3(ceil_div(n, NT), ceil_div(k, BAS_CH)), dim3(NT), 0, stream, n, N, k,
                     U, (const double *)W, P);
  POD2G_HIP_CHECK(hipGetLastError());
  std::vector<double> lh(N);
  POD2G_HIP_CHECK(hipMemcpyAsync(lh.data(), lam, sizeof(double) * N, hipMemcpyDeviceToHost, stream));
  POD2G_HIP_CHECK(hipStreamSynchronize(stream));
  if (!(lh[k - 1] > (double)N * 2.220446049250313e-16 * lh[0])) return POD2G_EINVAL;
  return POD2G_OK;
}

}  // extern "C"
