// FP64 kernels of the outer right-preconditioned FGMRES (restarted).
//
// Per iteration j (basis V_0..V_j orthonormal, z_j = M^{-1} V_j from the cycle):
//   k_apply_dot    w = H z_j (FP64), partial sums of h1_i = <V_i, w>
//   k_fin_sum      h1 = sum of partials (one block per value)
//   k_update_dot   w' = w - sum_i h1_i V_i, partial sums of h2_i = <V_i, w'> and ||w'||^2
//   k_fin_sum      h2, ||w'||^2
//   k_givens       H(:, j) = h1 + h2 (classical Gram-Schmidt with one re-orthogonalisation),
//                  h_{j+1,j}^2 = ||w'||^2 - ||h2||^2, Givens rotation of the Hessenberg
//                  column, residual estimate |g_{j+1}| / ||b||, convergence flag
//   k_normalize    V_{j+1} = (w' - sum_i h2_i V_i) / h_{j+1,j}
// Reductions are two-stage (per-block partials, then a fixed-order sum), so the
// results are bitwise reproducible run to run.
#include <cstddef>

#include "krylov.h"

namespace helm {

__device__ __forceinline__ cd wsum(cd v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

// sum v over the 256-thread block; thread 0 writes it to *out
__device__ __forceinline__ void block_sum(cd v, cd* lds, cd* out) {
  v = wsum(v);
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
}

__device__ __forceinline__ long long node_of(int q) {
  return ((long long)blockIdx.x * KNPT + q) * 256 + threadIdx.x;
}

template <typename CX>
__device__ __forceinline__ cd apply_h(const KrylovArgs& a, const CX* __restrict__ x, long long f) {
  const Geom& g = a.op.g;
  int i0 = (int)(f % g.N[0]);
  long long r = f / g.N[0];
  int i1 = (int)(r % g.N[1]), i2 = (int)(r / g.N[1]);
  double sig = layer_sigma(a.op, i0, i1, i2);
  double mm = a.m64[f];
  cd c = a.s * mk(mm, -mm * sig);
  if (a.conj) c.y = -c.y;
  cd D = mk(2.0 * g.dim * a.op.inv_h2 - c.x, -c.y);
  cd nb = mk(0.0, 0.0);
  long long s1 = g.N[0], s2 = (long long)g.N[0] * g.N[1];
  if (i0 > 0) nb += to_d(x[f - 1]);
  if (i0 < g.n[0]) nb += to_d(x[f + 1]);
  if (i1 > 0) nb += to_d(x[f - s1]);
  if (i1 < g.n[1]) nb += to_d(x[f + s1]);
  if (g.dim == 3) {
    if (i2 > 0) nb += to_d(x[f - s2]);
    if (i2 < g.n[2]) nb += to_d(x[f + s2]);
  }
  return D * to_d(x[f]) - a.op.inv_h2 * nb;
}

// w = H z (FP64), partials of <V_i, w> for i <= j
template <typename CZ>
__global__ void __launch_bounds__(256) k_apply_dot(KrylovArgs a, const CZ* __restrict__ z, int j) {
  __shared__ cd lds[4];
  const long long N = a.op.g.tot;
  cd w[KNPT];
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    w[q] = mk(0.0, 0.0);
    if (f < N) {
      w[q] = apply_h(a, z, f);
      a.W[f] = w[q];
    }
  }
  for (int i = 0; i <= j; ++i) {
    cd v = mk(0.0, 0.0);
    for (int q = 0; q < KNPT; ++q) {
      long long f = node_of(q);
      if (f < N) v += cmulc(a.V[(long long)i * a.ldv + f], w[q]);
    }
    block_sum(v, lds, a.part + (long long)i * a.pcap + blockIdx.x);
  }
}

// r = b - H x (FP64) into V_0; partials of (||r||^2, ||b||^2) in slot 0
__global__ void __launch_bounds__(256) k_residual(KrylovArgs a, const cd* __restrict__ x,
                                                  const cd* __restrict__ b) {
  __shared__ cd lds[4];
  const long long N = a.op.g.tot;
  cd v = mk(0.0, 0.0);
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f < N) {
      cd res = b[f] - apply_h(a, x, f);
      a.V[f] = res;
      v += mk(abs2(res), abs2(b[f]));
    }
  }
  block_sum(v, lds, a.part + blockIdx.x);
}

// one block per value: dst[i] = sum over blocks of part[i]
__global__ void __launch_bounds__(256) k_fin_sum(KrylovArgs a, cd* dst) {
  __shared__ cd lds[4];
  const int i = blockIdx.x;
  cd v = mk(0.0, 0.0);
  for (int b = threadIdx.x; b < a.nblk; b += 256) v += a.part[(long long)i * a.pcap + b];
  block_sum(v, lds, dst + i);
}

// w' = w - sum h1_i V_i ; partials of <V_i, w'> (i <= j) and ||w'||^2 (value j+1, .x)
__global__ void __launch_bounds__(256) k_update_dot(KrylovArgs a, int j) {
  __shared__ cd lds[4];
  __shared__ cd sh[KMAXM + 1];
  if (threadIdx.x <= j) sh[threadIdx.x] = a.st->h1[threadIdx.x];
  __syncthreads();
  const long long N = a.op.g.tot;
  cd w[KNPT];
  double nw = 0.0;
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    w[q] = mk(0.0, 0.0);
    if (f < N) {
      cd t = a.W[f];
      for (int i = 0; i <= j; ++i) t -= sh[i] * a.V[(long long)i * a.ldv + f];
      a.W[f] = t;
      w[q] = t;
      nw += abs2(t);
    }
  }
  for (int i = 0; i <= j; ++i) {
    cd v = mk(0.0, 0.0);
    for (int q = 0; q < KNPT; ++q) {
      long long f = node_of(q);
      if (f < N) v += cmulc(a.V[(long long)i * a.ldv + f], w[q]);
    }
    block_sum(v, lds, a.part + (long long)i * a.pcap + blockIdx.x);
  }
  block_sum(mk(nw, 0.0), lds, a.part + (long long)(j + 1) * a.pcap + blockIdx.x);
}

__device__ inline void givens(cd a, cd b, double& c, cd& s, cd& r) {
  double na = sqrt(abs2(a)), nb = sqrt(abs2(b));
  if (nb == 0.0) {
    c = 1.0; s = mk(0.0, 0.0); r = a;
    return;
  }
  if (na == 0.0) {
    c = 0.0; s = (1.0 / nb) * conjc(b); r = mk(nb, 0.0);
    return;
  }
  double t = hypot(na, nb);
  cd ph = (1.0 / na) * a;
  c = na / t;
  s = (1.0 / t) * (ph * conjc(b));
  r = t * ph;
}

// finish the Arnoldi column j and the Givens update (one thread)
__global__ void k_givens(KrylovArgs a, int j, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  KrylovState* st = a.st;
  const int ld = KMAXM + 1;
  double nw2 = st->h2[j + 1].x;
  double hh = 0.0;
  for (int i = 0; i <= j; ++i) {
    st->H[i + ld * j] = st->h1[i] + st->h2[i];
    hh += abs2(st->h2[i]);
  }
  double n2 = nw2 - hh;
  double hn = n2 > 0.0 ? sqrt(n2) : 0.0;
  st->H[j + 1 + ld * j] = mk(hn, 0.0);
  st->hnext = hn;
  for (int i = 0; i < j; ++i) {          // previous rotations on column j
    cd hi = st->H[i + ld * j], hi1 = st->H[i + 1 + ld * j];
    double c = st->cs[i];
    cd s = st->sn[i];
    st->H[i + ld * j] = c * hi + s * hi1;
    st->H[i + 1 + ld * j] = c * hi1 - conjc(s) * hi;
  }
  double c;
  cd s, r;
  givens(st->H[j + ld * j], st->H[j + 1 + ld * j], c, s, r);
  st->cs[j] = c;
  st->sn[j] = s;
  st->H[j + ld * j] = r;
  st->H[j + 1 + ld * j] = mk(0.0, 0.0);
  cd gj = st->g[j];
  st->g[j + 1] = -(conjc(s) * gj);
  st->g[j] = c * gj;
  double est = sqrt(abs2(st->g[j + 1])) / st->bnorm;
  st->est = est;
  if (st->its < KMAXIT) st->hist[st->its] = est;
  st->its += 1;
  bool fin = isfinite(est) && isfinite(hn);
  if (!fin) st->nonfinite = 1;
  st->done = (est <= tol || !fin || hn == 0.0) ? 1 : 0;
}

// V_{j+1} = (w' - sum h2_i V_i) / h_{j+1,j}
__global__ void __launch_bounds__(256) k_normalize(KrylovArgs a, int j) {
  __shared__ cd sh[KMAXM + 1];
  __shared__ double sinv;
  if (threadIdx.x <= j) sh[threadIdx.x] = a.st->h2[threadIdx.x];
  if (threadIdx.x == 0) sinv = a.st->hnext > 0.0 ? 1.0 / a.st->hnext : 0.0;
  __syncthreads();
  const long long N = a.op.g.tot;
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f >= N) continue;
    cd w = a.W[f];
    for (int i = 0; i <= j; ++i) w -= sh[i] * a.V[(long long)i * a.ldv + f];
    a.V[(long long)(j + 1) * a.ldv + f] = sinv * w;
  }
}

// restart bookkeeping from tmp = (||r||^2, ||b||^2): beta0, g = beta0 e1
__global__ void k_fin_residual(KrylovArgs a, int set_b) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  KrylovState* st = a.st;
  if (set_b) st->bnorm = sqrt(st->tmp[0].y);
  double b0 = sqrt(st->tmp[0].x);
  st->beta0 = b0;
  st->g[0] = mk(b0, 0.0);
  for (int i = 1; i <= KMAXM; ++i) st->g[i] = mk(0.0, 0.0);
  st->true_rel = st->bnorm > 0.0 ? b0 / st->bnorm : 0.0;
  st->done = 0;
  if (!isfinite(b0)) st->nonfinite = 1;
}

__global__ void __launch_bounds__(256) k_scale_v0(KrylovArgs a) {
  double s = a.st->beta0 > 0.0 ? 1.0 / a.st->beta0 : 0.0;
  const long long N = a.op.g.tot;
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f < N) a.V[f] = s * a.V[f];
  }
}

// y = R^{-1} g on the k x k upper triangle of the rotated Hessenberg matrix
__global__ void k_solve_y(KrylovArgs a, int k) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  KrylovState* st = a.st;
  const int ld = KMAXM + 1;
  for (int i = k - 1; i >= 0; --i) {
    cd acc = st->g[i];
    for (int l = i + 1; l < k; ++l) acc -= st->H[i + ld * l] * st->y[l];
    st->y[i] = cdiv(acc, st->H[i + ld * i]);
  }
}

// x += sum_i y_i Z_i
template <typename CZ>
__global__ void __launch_bounds__(256) k_update_x(KrylovArgs a, const CZ* __restrict__ Z, long long ldz, int k,
                                                  cd* __restrict__ x) {
  __shared__ cd sy[KMAXM];
  if (threadIdx.x < k) sy[threadIdx.x] = a.st->y[threadIdx.x];
  __syncthreads();
  const long long N = a.op.g.tot;
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f >= N) continue;
    cd acc = x[f];
    for (int i = 0; i < k; ++i) acc += sy[i] * to_d(Z[(long long)i * ldz + f]);
    x[f] = acc;
  }
}

__global__ void k_zero_c128(cd* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = mk(0.0, 0.0);
}

__global__ void k_init_state(KrylovState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->its = 0;
    st->nonfinite = 0;
    st->done = 0;
  }
}

// ------------------------------------------------------------- launchers ----
// device address of a cd array member of the (device-resident) state
static inline cd* st_field(const KrylovArgs& a, size_t off) { return (cd*)((char*)a.st + off); }

void kr_init(const KrylovArgs& a, hipStream_t s) { hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, a.st); }
void kr_residual(const KrylovArgs& a, const cd* x, const cd* b, int with_b, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(a.nblk), dim3(256), 0, s, a, x, b);
  hipLaunchKernelGGL(k_fin_sum, dim3(1), dim3(256), 0, s, a, st_field(a, offsetof(KrylovState, tmp)));
  hipLaunchKernelGGL(k_fin_residual, dim3(1), dim3(1), 0, s, a, with_b);
}
void kr_scale_v0(const KrylovArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_v0, dim3(a.nblk), dim3(256), 0, s, a);
}
void kr_arnoldi(const KrylovArgs& a, const void* z, int z_f32, int j, double tol, hipStream_t s) {
  dim3 g(a.nblk);
  if (z_f32)
    hipLaunchKernelGGL((k_apply_dot<cf>), g, dim3(256), 0, s, a, (const cf*)z, j);
  else
    hipLaunchKernelGGL((k_apply_dot<cd>), g, dim3(256), 0, s, a, (const cd*)z, j);
  hipLaunchKernelGGL(k_fin_sum, dim3(j + 1), dim3(256), 0, s, a, st_field(a, offsetof(KrylovState, h1)));
  hipLaunchKernelGGL(k_update_dot, g, dim3(256), 0, s, a, j);
  hipLaunchKernelGGL(k_fin_sum, dim3(j + 2), dim3(256), 0, s, a, st_field(a, offsetof(KrylovState, h2)));
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, s, a, j, tol);
  hipLaunchKernelGGL(k_normalize, g, dim3(256), 0, s, a, j);
}
void kr_update_x(const KrylovArgs& a, const void* Z, int z_f32, long long ldz, int k, cd* x, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_y, dim3(1), dim3(1), 0, s, a, k);
  dim3 g(a.nblk);
  if (z_f32)
    hipLaunchKernelGGL((k_update_x<cf>), g, dim3(256), 0, s, a, (const cf*)Z, ldz, k, x);
  else
    hipLaunchKernelGGL((k_update_x<cd>), g, dim3(256), 0, s, a, (const cd*)Z, ldz, k, x);
}
void kr_zero(cd* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_c128, dim3(1024), dim3(256), 0, s, x, n);
}

}  // namespace helm
