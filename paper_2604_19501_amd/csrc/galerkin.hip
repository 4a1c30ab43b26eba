// Galerkin coarse operators (setup, FP64).
//
//   A2 = R1 H_s P1          eq. (2.2), s = alpha2^2 (1 - i beta) omega^2
//   A3 = R2 (R1 H_s' P1) P2 eq. (3.6), s' = alpha^2 (1 - i beta) omega^2 (real shift, eq. (3.5))
//
// R is full weighting ([1 2 1]/4 per axis, truncated at the ends) and P = 2^d R^T
// (d-linear interpolation).  For every coarse node I the kernels form the row
//   A_c(I, J) = sum_f R(I, f) sum_g A(f, g) P(g, J),  J - I in {-1, 0, 1}^d,
// by walking the restriction footprint f, the fine stencil g = f + t and the
// (at most 2^d) interpolation parents J of g.  Output: 3^d complex coefficients
// per coarse node, structure of arrays, offset k = (d0+1) + 3 (d1+1) + 9 (d2+1).
#include "internal.h"

namespace helm {

__device__ __forceinline__ int koff(int dim, int d0, int d1, int d2) {
  return (d0 + 1) + 3 * (d1 + 1) + (dim == 3 ? 9 * (d2 + 1) : 0);
}

// accumulate a * P(g, J) into acc[J - I] over the parents J of fine node g
__device__ __forceinline__ void scatter_parents(int dim, const int* gI, const int* I, cd a, cd* acc) {
  int lo[3], hi[3];
  for (int q = 0; q < 3; ++q) {
    lo[q] = gI[q] >> 1;
    hi[q] = (gI[q] + 1) >> 1;
  }
  int nb2 = (dim == 3 && lo[2] != hi[2]) ? 2 : 1;
  int nb1 = lo[1] != hi[1] ? 2 : 1, nb0 = lo[0] != hi[0] ? 2 : 1;
  double w = 1.0;
  if (nb0 == 2) w *= 0.5;
  if (nb1 == 2) w *= 0.5;
  if (nb2 == 2) w *= 0.5;
  for (int b2 = 0; b2 < nb2; ++b2)
    for (int b1 = 0; b1 < nb1; ++b1)
      for (int b0 = 0; b0 < nb0; ++b0) {
        int J0 = b0 ? hi[0] : lo[0], J1 = b1 ? hi[1] : lo[1], J2 = b2 ? hi[2] : lo[2];
        int k = koff(dim, J0 - I[0], J1 - I[1], dim == 3 ? J2 - I[2] : 0);
        acc[k] += w * a;
      }
}

// a * P(g, J) into acc[J - I] for the parents J of the fine node g = 2 I + (d0, d1, d2),
// -2 <= d <= 2: along an axis an even d has the one parent I + d/2 (weight 1), an odd d
// the two parents I + (d -+ 1)/2 (weight 1/2 each).  Called from fully unrolled loops, so
// every index of acc is a constant and acc stays in registers.
template <int DIM>
__device__ __forceinline__ void add_parents(int d0, int d1, int d2, cd a, cd* acc) {
  const bool od0 = d0 & 1, od1 = d1 & 1, od2 = DIM == 3 && (d2 & 1);
  const double w = (od0 ? 0.5 : 1.0) * (od1 ? 0.5 : 1.0) * (od2 ? 0.5 : 1.0);
#pragma unroll
  for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
    for (int b1 = 0; b1 < 2; ++b1)
#pragma unroll
      for (int b0 = 0; b0 < 2; ++b0) {
        if ((od0 || !b0) && (od1 || !b1) && (od2 || !b2)) {
          const int J0 = od0 ? (b0 ? d0 + 1 : d0 - 1) / 2 : d0 / 2;
          const int J1 = od1 ? (b1 ? d1 + 1 : d1 - 1) / 2 : d1 / 2;
          const int J2 = DIM == 3 ? (od2 ? (b2 ? d2 + 1 : d2 - 1) / 2 : d2 / 2) : 0;
          acc[(J0 + 1) + 3 * (J1 + 1) + (DIM == 3 ? 9 * (J2 + 1) : 0)] += w * a;
        }
      }
}

// fine operator -Lap_h - s m (1 - i sigma) -> level 2.  Fine nodes outside the grid add
// zero terms, so the loops have constant trip counts.
template <int DIM>
__global__ void __launch_bounds__(128) k_gal_fine(FineOp op, cd s, const double* __restrict__ m,
                                                  Geom gc, cd* __restrict__ out) {
  constexpr int R2 = DIM == 3 ? 1 : 0, K = DIM == 3 ? 27 : 9;
  long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= gc.tot) return;
  const Geom& g = op.g;
  const int Ic[3] = {(int)(I % gc.N[0]), (int)((I / gc.N[0]) % gc.N[1]),
                     DIM == 3 ? (int)(I / ((long long)gc.N[0] * gc.N[1])) : 0};
  cd acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = mk(0.0, 0.0);
  const double ih = op.inv_h2;
#pragma unroll
  for (int o2 = -R2; o2 <= R2; ++o2)
#pragma unroll
    for (int o1 = -1; o1 <= 1; ++o1)
#pragma unroll
      for (int o0 = -1; o0 <= 1; ++o0) {
        const int f[3] = {2 * Ic[0] + o0, 2 * Ic[1] + o1, 2 * Ic[2] + o2};
        const bool in = f[0] >= 0 && f[0] <= g.n[0] && f[1] >= 0 && f[1] <= g.n[1] &&
                        (DIM == 2 || (f[2] >= 0 && f[2] <= g.n[2]));
        const double wR = (o0 == 0 ? 0.5 : 0.25) * (o1 == 0 ? 0.5 : 0.25) * (DIM == 3 ? (o2 == 0 ? 0.5 : 0.25) : 1.0);
        cd diag = mk(0.0, 0.0);
        if (in) {
          const long long fl = f[0] + (long long)g.N[0] * (f[1] + (long long)g.N[1] * f[2]);
          const double sig = layer_sigma(op, f[0], f[1], f[2]);
          const double mm = m[fl];
          const cd c = s * mk(mm, -mm * sig);
          diag = mk(2.0 * DIM * ih - c.x, -c.y);
        }
        add_parents<DIM>(o0, o1, o2, wR * diag, acc);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int sgn = -1; sgn <= 1; sgn += 2) {
            const int ga = f[a] + sgn;
            const bool ing = in && ga >= 0 && ga <= g.n[a];
            add_parents<DIM>(o0 + (a == 0 ? sgn : 0), o1 + (a == 1 ? sgn : 0), o2 + (a == 2 ? sgn : 0),
                             ing ? mk(-wR * ih, 0.0) : mk(0.0, 0.0), acc);
          }
      }
#pragma unroll
  for (int k = 0; k < K; ++k) out[(long long)k * gc.tot + I] = acc[k];
}

// stored 3^d operator on level 2 -> level 3
__global__ void __launch_bounds__(128) k_gal_coarse(Geom g, const cd* __restrict__ A, Geom gc,
                                                    cd* __restrict__ out) {
  long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= gc.tot) return;
  int dim = g.dim;
  int Ic[3] = {(int)(I % gc.N[0]), (int)((I / gc.N[0]) % gc.N[1]), (int)(I / ((long long)gc.N[0] * gc.N[1]))};
  cd acc[27];
  for (int k = 0; k < 27; ++k) acc[k] = mk(0.0, 0.0);
  int r2 = dim == 3 ? 1 : 0;
  for (int o2 = -r2; o2 <= r2; ++o2)
    for (int o1 = -1; o1 <= 1; ++o1)
      for (int o0 = -1; o0 <= 1; ++o0) {
        int f[3] = {2 * Ic[0] + o0, 2 * Ic[1] + o1, dim == 3 ? 2 * Ic[2] + o2 : 0};
        if (f[0] < 0 || f[0] > g.n[0] || f[1] < 0 || f[1] > g.n[1] || f[2] < 0 || f[2] > g.n[2]) continue;
        double wR = (o0 == 0 ? 0.5 : 0.25) * (o1 == 0 ? 0.5 : 0.25) * (dim == 3 ? (o2 == 0 ? 0.5 : 0.25) : 1.0);
        long long fl = f[0] + (long long)g.N[0] * (f[1] + (long long)g.N[1] * f[2]);
        for (int t2 = -r2; t2 <= r2; ++t2)
          for (int t1 = -1; t1 <= 1; ++t1)
            for (int t0 = -1; t0 <= 1; ++t0) {
              int gI[3] = {f[0] + t0, f[1] + t1, f[2] + t2};
              if (gI[0] < 0 || gI[0] > g.n[0] || gI[1] < 0 || gI[1] > g.n[1] || gI[2] < 0 || gI[2] > g.n[2])
                continue;
              cd a = A[(long long)koff(dim, t0, t1, t2) * g.tot + fl];
              scatter_parents(dim, gI, Ic, wR * a, acc);
            }
      }
  int K = dim == 3 ? 27 : 9;
  for (int k = 0; k < K; ++k) out[(long long)k * gc.tot + I] = acc[k];
}

__global__ void k_cast_d2f(const cd* __restrict__ a, cf* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = to_f(a[i]);
}

// m = kappa^2 from the slowness (is_m = 0), or m taken as given (is_m = 1)
__global__ void k_square(const double* __restrict__ kap, double* __restrict__ m64, float* __restrict__ m32,
                         long long n, int is_m) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double v = is_m ? kap[i] : kap[i] * kap[i];
    m64[i] = v;
    m32[i] = (float)v;
  }
}

void gal_fine(const FineOp& op, cd s, const double* m, const Geom& gc, cd* out, hipStream_t st) {
  const dim3 grid((unsigned)((gc.tot + 127) / 128));
  if (op.g.dim == 3)
    hipLaunchKernelGGL(k_gal_fine<3>, grid, dim3(128), 0, st, op, s, m, gc, out);
  else
    hipLaunchKernelGGL(k_gal_fine<2>, grid, dim3(128), 0, st, op, s, m, gc, out);
}
void gal_coarse(const Geom& g, const cd* A, const Geom& gc, cd* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gal_coarse, dim3((unsigned)((gc.tot + 127) / 128)), dim3(128), 0, st, g, A, gc, out);
}
void cast_d2f(const cd* a, cf* b, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(1024), dim3(256), 0, st, a, b, n);
}
void square_slowness(const double* kap, double* m64, float* m32, long long n, int is_m, hipStream_t st) {
  hipLaunchKernelGGL(k_square, dim3(1024), dim3(256), 0, st, kap, m64, m32, n, is_m);
}

}  // namespace helm
