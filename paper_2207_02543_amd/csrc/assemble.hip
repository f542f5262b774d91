// Pattern, element matrix and assembly of K(theta), D^-1 and f
// (Sec. 2.1, Eqs. 5-6): gathered per stored entry, deterministic.
#include "common.hpp"

#include <math.h>

namespace pod2g {

template <int DIM>
__device__ __forceinline__ void node_coords(int N, int node, int &i, int &j, int &l) {
  if (DIM == 2) {
    i = node % N + 1;
    j = node / N;
    l = 0;
  } else {
    const int np = N + 1;
    i = node % np;
    j = (node / np) % np;
    l = node / (np * np) + 1;
  }
}

// Free-node rank of (i,j,l), or -1 if outside the mesh or clamped.
template <int DIM>
__device__ __forceinline__ int node_rank(int N, int i, int j, int l) {
  if (i < 0 || i > N || j < 0 || j > N) return -1;
  if (DIM == 2) return i >= 1 ? (i - 1) + N * j : -1;
  if (l < 1 || l > N) return -1;
  return i + (N + 1) * j + (N + 1) * (N + 1) * (l - 1);
}

template <int DIM>
__global__ void __launch_bounds__(NT) k_pattern(int N, int nn, int *__restrict__ colblk) {
  const int node = blockIdx.x * NT + threadIdx.x;
  if (node >= nn) return;
  int i, j, l;
  node_coords<DIM>(N, node, i, j, l);
  for (int s = 0; s < Stencil<DIM>::S; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = DIM == 3 ? s / 9 - 1 : 0;
    const int nb = node_rank<DIM>(N, i + dx, j + dy, l + dz);
    colblk[s * nn + node] = nb >= 0 ? nb : node;
  }
}

// Unit-modulus element matrix by 2^DIM-point Gauss quadrature:
// K[p][q] = sum_g det(J) eps_p^T D eps_q, eps_p the strain of a unit
// displacement of element DOF p (engineering shear).  One thread per entry
// of the upper triangle; the lower one is its mirror (exactly symmetric).
template <int DIM>
__global__ void k_kref(double nu, double h, double *__restrict__ kref) {
  constexpr int ED = Stencil<DIM>::ED;
  const int t = threadIdx.x;
  if (t >= ED * ED) return;
  int p = t / ED, q = t % ED;
  const bool mirror = p > q;
  if (mirror) { const int tmp = p; p = q; q = tmp; }
  const int lp = p / DIM, cp = p % DIM, lq = q / DIM, cq = q % DIM;
  const double g = 1.0 / sqrt(3.0);
  const double detJ = DIM == 2 ? (h / 2) * (h / 2) : (h / 2) * (h / 2) * (h / 2);
  double acc = 0.0;
  for (int gp = 0; gp < (1 << DIM); ++gp) {
    double xi[3];
    for (int d = 0; d < DIM; ++d) xi[d] = ((gp >> d) & 1) ? g : -g;
    double gradp[3], gradq[3];
    for (int d = 0; d < DIM; ++d) {
      double vp = (double)(2 * ((lp >> d) & 1) - 1), vq = (double)(2 * ((lq >> d) & 1) - 1);
      double wp = vp, wq = vq;
      for (int e = 0; e < DIM; ++e) {
        if (e == d) continue;
        wp *= 1.0 + (double)(2 * ((lp >> e) & 1) - 1) * xi[e];
        wq *= 1.0 + (double)(2 * ((lq >> e) & 1) - 1) * xi[e];
      }
      gradp[d] = wp / (double)(1 << DIM) * (2.0 / h);
      gradq[d] = wq / (double)(1 << DIM) * (2.0 / h);
    }
    if (DIM == 2) {
      // strains (xx, yy, xy) of the unit displacements
      const double ep[3] = {cp == 0 ? gradp[0] : 0.0, cp == 1 ? gradp[1] : 0.0,
                            cp == 0 ? gradp[1] : gradp[0]};
      const double eq[3] = {cq == 0 ? gradq[0] : 0.0, cq == 1 ? gradq[1] : 0.0,
                            cq == 0 ? gradq[1] : gradq[0]};
      const double c = 1.0 / (1.0 - nu * nu);
      const double De0 = c * (eq[0] + nu * eq[1]);
      const double De1 = c * (nu * eq[0] + eq[1]);
      const double De2 = c * 0.5 * (1.0 - nu) * eq[2];
      acc += detJ * (ep[0] * De0 + ep[1] * De1 + ep[2] * De2);
    } else {
      double ep[6] = {0, 0, 0, 0, 0, 0}, eq[6] = {0, 0, 0, 0, 0, 0};
      ep[cp] = gradp[cp];
      eq[cq] = gradq[cq];
      // shear strains xy, yz, zx
      if (cp == 0) { ep[3] = gradp[1]; ep[5] = gradp[2]; }
      if (cp == 1) { ep[3] = gradp[0]; ep[4] = gradp[2]; }
      if (cp == 2) { ep[4] = gradp[1]; ep[5] = gradp[0]; }
      if (cq == 0) { eq[3] = gradq[1]; eq[5] = gradq[2]; }
      if (cq == 1) { eq[3] = gradq[0]; eq[4] = gradq[2]; }
      if (cq == 2) { eq[4] = gradq[1]; eq[5] = gradq[0]; }
      const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
      const double mu = 1.0 / (2.0 * (1.0 + nu));
      const double tr = eq[0] + eq[1] + eq[2];
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += ep[a] * (lam * tr + 2.0 * mu * eq[a]);
      for (int a = 3; a < 6; ++a) s += ep[a] * (mu * eq[a]);
      acc += detJ * s;
    }
  }
  kref[threadIdx.x] = acc;
  (void)mirror;
}

// Element moduli: E = exp(kl_scale * sum_t xi_t prod_d cos(pi a_td c_d) / (1 + |a_t|)).
// The t-th multi-index is the base-4 digit string of t + 1 (x most significant).
template <int DIM>
__global__ void __launch_bounds__(NT) k_young(int N, int ne, int n_terms, double kl_scale,
                                              const double *__restrict__ xi, double *__restrict__ E) {
  const int e = blockIdx.x * NT + threadIdx.x;
  const int b = blockIdx.y;
  if (e >= ne) return;
  const double h = 1.0 / N;
  int ec[3] = {e % N, (e / N) % N, DIM == 3 ? e / (N * N) : 0};
  double c[3];
  for (int d = 0; d < DIM; ++d) c[d] = (ec[d] + 0.5) * h;
  const double *x = xi + (size_t)b * n_terms;
  double g = 0.0;
  for (int t = 0; t < n_terms; ++t) {
    int code = t + 1;
    int a[3];
    for (int d = DIM - 1; d >= 0; --d) { a[d] = code & 3; code >>= 2; }
    double term = 1.0;
    int asum = 0;
    for (int d = 0; d < DIM; ++d) {
      term = term * cos(M_PI * (double)a[d] * c[d]);
      asum += a[d];
    }
    g += x[t] * term / (1.0 + (double)asum);
  }
  E[(size_t)b * ne + e] = exp(kl_scale * g);
}

// One thread per scalar row: the row's stored values (centre and upper
// slots of the symmetric half storage; see Half in common.hpp); the first
// DIM threads also clear the zero node of every plane.
template <int DIM>
__global__ void __launch_bounds__(NT) k_assemble(int N, int n, int nn, int ne, long long vstride,
                                                 const double *__restrict__ E,
                                                 const double *__restrict__ kref,
                                                 double *__restrict__ vals, float *__restrict__ vals32,
                                                 double *__restrict__ dinv) {
  constexpr int ED = Stencil<DIM>::ED;
  constexpr int S = Stencil<DIM>::S;
  __shared__ double sk[ED * ED];
  for (int t = threadIdx.x; t < ED * ED; t += NT) sk[t] = kref[t];
  __syncthreads();
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  const int b = blockIdx.y;
  const double *Eb = E + (size_t)b * ne;
  double *vb = vals + (size_t)b * vstride;
  float *v32 = vals32 ? vals32 + (size_t)b * vstride : nullptr;
  const int node = row / DIM, a = row % DIM;
  const size_t ns = (size_t)n + DIM;
  constexpr int H = Half<DIM>::H;
  if (row < DIM)
    for (int p = 0; p < Half<DIM>::SH * DIM; ++p) {
      vb[(size_t)p * ns + n + row] = 0.0;
      if (v32) v32[(size_t)p * ns + n + row] = 0.f;
    }
  int ci[3];
  node_coords<DIM>(N, node, ci[0], ci[1], ci[2]);
  for (int s = H; s < S; ++s) {
    const int dd[3] = {s % 3 - 1, (s / 3) % 3 - 1, DIM == 3 ? s / 9 - 1 : 0};
    const int nb = node_rank<DIM>(N, ci[0] + dd[0], ci[1] + dd[1], ci[2] + dd[2]);
    double acc[DIM];
    for (int bc = 0; bc < DIM; ++bc) acc[bc] = 0.0;
    if (nb >= 0) {
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        if (d >= DIM) { lo[d] = hi[d] = 0; continue; }
        const int m = ci[d] + dd[d];
        lo[d] = (ci[d] > m ? ci[d] : m) - 1;
        hi[d] = ci[d] < m ? ci[d] : m;
        if (lo[d] < 0) lo[d] = 0;
        if (hi[d] > N - 1) hi[d] = N - 1;
      }
      for (int ez = lo[2]; ez <= hi[2]; ++ez)
        for (int ey = lo[1]; ey <= hi[1]; ++ey)
          for (int ex = lo[0]; ex <= hi[0]; ++ex) {
            const int el = ex + N * ey + (DIM == 3 ? N * N * ez : 0);
            const int lr = (ci[0] - ex) + 2 * (ci[1] - ey) + (DIM == 3 ? 4 * (ci[2] - ez) : 0);
            const int lc = (ci[0] + dd[0] - ex) + 2 * (ci[1] + dd[1] - ey) +
                           (DIM == 3 ? 4 * (ci[2] + dd[2] - ez) : 0);
            const double Ee = Eb[el];
            const double *krow = sk + (DIM * lr + a) * ED + DIM * lc;
            for (int bc = 0; bc < DIM; ++bc) acc[bc] += Ee * krow[bc];
          }
    }
    for (int bc = 0; bc < DIM; ++bc) {
      const size_t idx = (size_t)((s - H) * DIM + bc) * ns + row;
      vb[idx] = acc[bc];
      if (v32) v32[idx] = (float)acc[bc];
    }
    if (s == H) dinv[(size_t)b * n + row] = 1.0 / acc[a];
  }
}

// Consistent nodal forces of the unit traction (+x on x = 1 in 2D, +z on z = 1 in 3D).
template <int DIM>
__global__ void __launch_bounds__(NT) k_traction(int N, int n, double *__restrict__ f) {
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  const int node = row / DIM, a = row % DIM;
  int i, j, l;
  node_coords<DIM>(N, node, i, j, l);
  const double h = 1.0 / N;
  double v = 0.0;
  if (DIM == 2) {
    if (i == N && a == 0) v = (j == 0 || j == N) ? h / 2 : h;
  } else {
    if (l == N && a == 2) {
      const int cx = (i == 0 || i == N) ? 1 : 2, cy = (j == 0 || j == N) ? 1 : 2;
      v = (double)(cx * cy) * (h * h / 4);
    }
  }
  f[row] = v;
}

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static int check_mesh(const pod2g_mesh *m) {
  if (!m) return POD2G_EINVAL;
  if (m->dim != 2 && m->dim != 3) return POD2G_EINVAL;
  if (m->N < 1 || m->N > 4096) return POD2G_EINVAL;
  const int maxterms = m->dim == 2 ? 15 : 63;
  if (m->n_terms < 1 || m->n_terms > maxterms) return POD2G_EINVAL;
  if (!(m->nu >= 0.0 && m->nu < 0.5)) return POD2G_EINVAL;
  const long long N = m->N;
  const long long nn = m->dim == 2 ? N * (N + 1) : (N + 1) * (N + 1) * N;
  const long long nvals = nn * m->dim * (m->dim == 2 ? 9 : 27) * m->dim;
  if (nvals >= (1ll << 31)) return POD2G_EINVAL;
  return POD2G_OK;
}

}  // namespace pod2g

using namespace pod2g;

extern "C" {

size_t pod2g_pattern_bytes(const pod2g_mesh *m) {
  if (check_mesh(m) != POD2G_OK) return 0;
  const long long N = m->N;
  const long long nn = m->dim == 2 ? N * (N + 1) : (N + 1) * (N + 1) * N;
  const int S = m->dim == 2 ? 9 : 27, ED = m->dim * (1 << m->dim);
  return align256((size_t)S * nn * sizeof(int)) + align256((size_t)ED * ED * sizeof(double));
}

int pod2g_pattern_build(const pod2g_mesh *m, void *dbuf, size_t bytes, pod2g_pattern *out,
                        hipStream_t stream) {
  int st = check_mesh(m);
  if (st) return st;
  if (!dbuf || !out) return POD2G_EINVAL;
  if (bytes < pod2g_pattern_bytes(m)) return POD2G_ESIZE;
  const int N = m->N, dim = m->dim;
  pod2g_pattern p;
  p.mesh = *m;
  p.n_nodes = dim == 2 ? N * (N + 1) : (N + 1) * (N + 1) * N;
  p.n = dim * p.n_nodes;
  p.n_slots = dim == 2 ? 9 : 27;
  p.n_elems = dim == 2 ? N * N : N * N * N;
  p.nvals = (long long)(p.n + dim) * (p.n_slots / 2 + 1) * dim;   // symmetric half storage
  p.colblk = (int *)dbuf;
  p.kref = (double *)((char *)dbuf + align256((size_t)p.n_slots * p.n_nodes * sizeof(int)));
  const int ED = dim * (1 << dim);
  const double h = 1.0 / N;
  if (dim == 2) {
    hipLaunchKernelGGL(k_pattern<2>, dim3(ceil_div(p.n_nodes, NT)), dim3(NT), 0, stream, N,
                       p.n_nodes, p.colblk);
    hipLaunchKernelGGL(k_kref<2>, dim3(1), dim3(ED * ED), 0, stream, m->nu, h, p.kref);
  } else {
    hipLaunchKernelGGL(k_pattern<3>, dim3(ceil_div(p.n_nodes, NT)), dim3(NT), 0, stream, N,
                       p.n_nodes, p.colblk);
    hipLaunchKernelGGL(k_kref<3>, dim3(1), dim3(ED * ED), 0, stream, m->nu, h, p.kref);
  }
  POD2G_HIP_CHECK(hipGetLastError());
  *out = p;
  return POD2G_OK;
}

size_t pod2g_assemble_bytes(const pod2g_pattern *pat, int batch) {
  if (!pat || batch < 1) return 0;
  return align256((size_t)batch * pat->n_elems * sizeof(double));
}

int pod2g_assemble(const pod2g_pattern *pat, const double *xi, int batch, double *vals,
                   float *vals32, double *dinv, double *f, void *work, size_t bytes,
                   hipStream_t stream) {
  if (!pat || !xi || !vals || !dinv || !work || batch < 1 || batch > 65535) return POD2G_EINVAL;
  if (check_mesh(&pat->mesh)) return POD2G_EINVAL;
  if (bytes < pod2g_assemble_bytes(pat, batch)) return POD2G_ESIZE;
  const pod2g_mesh &m = pat->mesh;
  double *E = (double *)work;
  dim3 gy(ceil_div(pat->n_elems, NT), batch), ga(ceil_div(pat->n, NT), batch);
  if (m.dim == 2) {
    hipLaunchKernelGGL(k_young<2>, gy, dim3(NT), 0, stream, m.N, pat->n_elems, m.n_terms,
                       m.kl_scale, xi, E);
    hipLaunchKernelGGL(k_assemble<2>, ga, dim3(NT), 0, stream, m.N, pat->n, pat->n_nodes,
                       pat->n_elems, pat->nvals, E, pat->kref, vals, vals32, dinv);
    if (f) hipLaunchKernelGGL(k_traction<2>, dim3(ceil_div(pat->n, NT)), dim3(NT), 0, stream, m.N, pat->n, f);
  } else {
    hipLaunchKernelGGL(k_young<3>, gy, dim3(NT), 0, stream, m.N, pat->n_elems, m.n_terms,
                       m.kl_scale, xi, E);
    hipLaunchKernelGGL(k_assemble<3>, ga, dim3(NT), 0, stream, m.N, pat->n, pat->n_nodes,
                       pat->n_elems, pat->nvals, E, pat->kref, vals, vals32, dinv);
    if (f) hipLaunchKernelGGL(k_traction<3>, dim3(ceil_div(pat->n, NT)), dim3(NT), 0, stream, m.N, pat->n, f);
  }
  POD2G_HIP_CHECK(hipGetLastError());
  return POD2G_OK;
}

}  // extern "C"
