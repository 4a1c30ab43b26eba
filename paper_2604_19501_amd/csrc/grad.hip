// Gradient of the least-squares misfit w.r.t. squared slowness, and precision casts.
//
// With H(m) = -Lap_h - omega^2 m (1 - i sigma) (eq. (1.1) with the absorbing
// layer), dH/dm_j = -omega^2 (1 - i sigma_j) e_j e_j^T, so for H u = q and the
// adjoint field H^H lambda = P^T (P u - d) the misfit derivative is
//     g_j = omega^2 Re( conj(lambda_j) (1 - i sigma_j) u_j ),
// summed over sources.
#include "internal.h"

namespace helm {

__global__ void __launch_bounds__(256) k_grad(FineOp op, double w2, const cd* __restrict__ u,
                                              const cd* __restrict__ lam, double* __restrict__ g, int first) {
  const Geom& G = op.g;
  for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < G.tot;
       f += (long long)gridDim.x * blockDim.x) {
    int i0 = (int)(f % G.N[0]);
    long long r = f / G.N[0];
    int i1 = (int)(r % G.N[1]), i2 = (int)(r / G.N[1]);
    double sig = layer_sigma(op, i0, i1, i2);
    cd t = mk(1.0, -sig) * u[f];           // (1 - i sigma) u
    double v = w2 * (lam[f].x * t.x + lam[f].y * t.y);   // Re(conj(lambda) t)
    g[f] = first ? v : g[f] + v;
  }
}

__global__ void k_cast_f2d(const cf* __restrict__ a, cd* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = to_d(a[i]);
}

void grad_accumulate(const FineOp& op, double omega, const cd* u, const cd* lam, double* g, int first,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_grad, dim3(2048), dim3(256), 0, s, op, omega * omega, u, lam, g, first);
}
void cast_f2d(const cf* a, cd* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f2d, dim3(1024), dim3(256), 0, s, a, b, n);
}

}  // namespace helm
