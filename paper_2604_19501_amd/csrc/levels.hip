// Stencil kernels of the multigrid cycle on levels 1 and 2 (gfx950).
//
// Level 1 is the 5-point (2D) / 7-point (3D) operator of eq. (1.1) with the
// absorbing layer, H_s = -Lap_h - s m (1 - i sigma), evaluated on the fly from
// the squared slowness m (sigma is analytic in the node index).  Level 2 is the
// Galerkin operator of eq. (2.2), stored as 9 / 27 complex coefficients per node
// (structure of arrays: coefficient k of node i at coef[k*N + i]).
//
// Every relaxation / restriction kernel evaluates its input iterate "virtually":
//     x_in = [stored x] + [omega D^{-1} b, the first Jacobi sweep from zero]
//                       + [P e, the coarse-grid correction]
// so the first sweep, the correction and the following sweep are fused into one
// pass (the two-grid algorithm of Sec. 2 without materialising intermediate
// iterates).  Damped Jacobi:  x_out = x_in + w D^{-1} (b - A x_in).
//
// Threads map to nodes x-fastest (coalesced); blocks are remapped so that each
// of the 8 XCDs sweeps a contiguous slab, keeping neighbour planes in its L2.
#include "levels_api.h"

namespace helm {



// contiguous-slab block order: hardware dispatches block b to XCD b % 8
__device__ __forceinline__ long long xcd_block(long long nblocks) {
  long long b = blockIdx.x;
  long long per = (nblocks + 7) / 8;
  long long xcd = b % 8, k = b / 8;
  long long lb = xcd * per + k;
  return lb;   // may exceed nblocks - 1: caller bounds-checks the node index
}

__device__ __forceinline__ void decode(const Geom& g, long long f, int& i0, int& i1, int& i2) {
  i0 = (int)(f % g.N[0]);
  long long r = f / g.N[0];
  i1 = (int)(r % g.N[1]);
  i2 = (int)(r / g.N[1]);
}

// P e at fine node (i0,i1,i2): d-linear interpolation of the coarse vector e
template <typename C>
__device__ __forceinline__ C prolong_at(const Geom& gc, const C* __restrict__ e, int i0, int i1, int i2,
                                        int dim) {
  int lo[3], hi[3];
  int ii[3] = {i0, i1, i2};
  for (int a = 0; a < 3; ++a) {
    lo[a] = ii[a] >> 1;
    hi[a] = (ii[a] + 1) >> 1;
  }
  C acc = mk((decltype(acc.x))0, (decltype(acc.x))0);
  typedef decltype(acc.x) R;
  if (dim == 2) {
    R w0 = (lo[0] == hi[0]) ? (R)1 : (R)0.5, w1 = (lo[1] == hi[1]) ? (R)1 : (R)0.5;
    for (int b1 = 0; b1 < (lo[1] == hi[1] ? 1 : 2); ++b1)
      for (int b0 = 0; b0 < (lo[0] == hi[0] ? 1 : 2); ++b0) {
        int c0 = b0 ? hi[0] : lo[0], c1 = b1 ? hi[1] : lo[1];
        acc += (w0 * w1) * e[c0 + (long long)gc.N[0] * c1];
      }
  } else {
    R w0 = (lo[0] == hi[0]) ? (R)1 : (R)0.5, w1 = (lo[1] == hi[1]) ? (R)1 : (R)0.5,
      w2 = (lo[2] == hi[2]) ? (R)1 : (R)0.5;
    for (int b2 = 0; b2 < (lo[2] == hi[2] ? 1 : 2); ++b2)
      for (int b1 = 0; b1 < (lo[1] == hi[1] ? 1 : 2); ++b1)
        for (int b0 = 0; b0 < (lo[0] == hi[0] ? 1 : 2); ++b0) {
          int c0 = b0 ? hi[0] : lo[0], c1 = b1 ? hi[1] : lo[1], c2 = b2 ? hi[2] : lo[2];
          acc += (w0 * w1 * w2) * e[c0 + (long long)gc.N[0] * (c1 + (long long)gc.N[1] * c2)];
        }
  }
  return acc;
}

// virtual iterate at a level-1 node
template <typename R, typename CB, int XIN>
__device__ __forceinline__ typename cplx<R>::type xin_l1(const L1<R>& A, const typename cplx<R>::type* __restrict__ x,
                                                        const CB* __restrict__ b, R w, const Geom& gc,
                                                        const typename cplx<R>::type* __restrict__ e,
                                                        long long f, int i0, int i1, int i2) {
  typedef typename cplx<R>::type C;
  C v = mk((R)0, (R)0);
  if (XIN & XIN_X) v += x[f];
  if (XIN & XIN_Z) {
    C d = A.diag(f, i0, i1, i2);
    v += w * cdiv(conv<C>::from(b[f]), d);
  }
  if (XIN & XIN_E) v += prolong_at(gc, e, i0, i1, i2, A.op.g.dim);
  return v;
}

// (A x_in)(f) and D(f) for the level-1 operator
template <typename R, typename CB, int XIN>
__device__ __forceinline__ void apply_l1(const L1<R>& A, const typename cplx<R>::type* __restrict__ x,
                                         const CB* __restrict__ b, R w, const Geom& gc,
                                         const typename cplx<R>::type* __restrict__ e, long long f, int i0,
                                         int i1, int i2, typename cplx<R>::type& Ax,
                                         typename cplx<R>::type& xc, typename cplx<R>::type& D) {
  typedef typename cplx<R>::type C;
  const Geom& g = A.op.g;
  D = A.diag(f, i0, i1, i2);
  xc = xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f, i0, i1, i2);
  C nb = mk((R)0, (R)0);
  long long s1 = g.N[0], s2 = (long long)g.N[0] * g.N[1];
  if (i0 > 0) nb += xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f - 1, i0 - 1, i1, i2);
  if (i0 < g.n[0]) nb += xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f + 1, i0 + 1, i1, i2);
  if (i1 > 0) nb += xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f - s1, i0, i1 - 1, i2);
  if (i1 < g.n[1]) nb += xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f + s1, i0, i1 + 1, i2);
  if (g.dim == 3) {
    if (i2 > 0) nb += xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f - s2, i0, i1, i2 - 1);
    if (i2 < g.n[2]) nb += xin_l1<R, CB, XIN>(A, x, b, w, gc, e, f + s2, i0, i1, i2 + 1);
  }
  R ih = (R)A.op.inv_h2;
  Ax = D * xc - ih * nb;
}

// x_out = x_in + w D^{-1}(b - A x_in)   (w = 0: just materialise x_in)
template <typename R, typename CB, typename CO, int XIN>
__global__ void __launch_bounds__(256) k_l1_sweep(L1<R> A, const typename cplx<R>::type* __restrict__ x,
                                                  const CB* __restrict__ b, R w_in, Geom gc,
                                                  const typename cplx<R>::type* __restrict__ e, R w,
                                                  CO* __restrict__ out) {
  typedef typename cplx<R>::type C;
  const Geom& g = A.op.g;
  long long nb = (g.tot + 255) / 256;
  long long f = xcd_block(nb) * 256 + threadIdx.x;
  if (f >= g.tot) return;
  int i0, i1, i2;
  decode(g, f, i0, i1, i2);
  C Ax, xc, D;
  apply_l1<R, CB, XIN>(A, x, b, w_in, gc, e, f, i0, i1, i2, Ax, xc, D);
  C r = conv<C>::from(b[f]) - Ax;
  C y = xc + w * cdiv(r, D);
  out[f] = conv<CO>::from(y);
}

// b2(I) = sum_f R(I, f) (b - A x_in)(f), full weighting [1 2 1]/4 per axis
template <typename R, typename CB, int XIN>
__global__ void __launch_bounds__(256) k_l1_restrict(L1<R> A, const typename cplx<R>::type* __restrict__ x,
                                                     const CB* __restrict__ b, R w_in, Geom gc,
                                                     const typename cplx<R>::type* __restrict__ e,
                                                     Geom g2, typename cplx<R>::type* __restrict__ b2) {
  typedef typename cplx<R>::type C;
  const Geom& g = A.op.g;
  long long nb = (g2.tot + 255) / 256;
  long long I = xcd_block(nb) * 256 + threadIdx.x;
  if (I >= g2.tot) return;
  int I0, I1, I2;
  decode(g2, I, I0, I1, I2);
  C acc = mk((R)0, (R)0);
  int r2 = g.dim == 3 ? 1 : 0;
  for (int o2 = -r2; o2 <= r2; ++o2) {
    int f2 = 2 * I2 + o2;
    if (f2 < 0 || f2 > g.n[2]) continue;
    R w2 = (g.dim == 3) ? (o2 == 0 ? (R)0.5 : (R)0.25) : (R)1;
    for (int o1 = -1; o1 <= 1; ++o1) {
      int f1 = 2 * I1 + o1;
      if (f1 < 0 || f1 > g.n[1]) continue;
      R w1 = o1 == 0 ? (R)0.5 : (R)0.25;
      for (int o0 = -1; o0 <= 1; ++o0) {
        int f0 = 2 * I0 + o0;
        if (f0 < 0 || f0 > g.n[0]) continue;
        R w0 = o0 == 0 ? (R)0.5 : (R)0.25;
        long long f = f0 + (long long)g.N[0] * (f1 + (long long)g.N[1] * f2);
        C Ax, xc, D;
        apply_l1<R, CB, XIN>(A, x, b, w_in, gc, e, f, f0, f1, f2, Ax, xc, D);
        C r = conv<C>::from(b[f]) - Ax;
        acc += (w0 * w1 * w2) * r;
      }
    }
  }
  b2[I] = acc;
}

// y = A x for the outer operator (FP64 arithmetic), x in c64 or c128
template <typename CX>
__global__ void __launch_bounds__(256) k_l1_apply64(L1<double> A, const CX* __restrict__ x,
                                                    cd* __restrict__ y) {
  const Geom& g = A.op.g;
  long long nb = (g.tot + 255) / 256;
  long long f = xcd_block(nb) * 256 + threadIdx.x;
  if (f >= g.tot) return;
  int i0, i1, i2;
  decode(g, f, i0, i1, i2);
  cd D = A.diag(f, i0, i1, i2);
  cd nbs = mk(0.0, 0.0);
  long long s1 = g.N[0], s2 = (long long)g.N[0] * g.N[1];
  if (i0 > 0) nbs += to_d(x[f - 1]);
  if (i0 < g.n[0]) nbs += to_d(x[f + 1]);
  if (i1 > 0) nbs += to_d(x[f - s1]);
  if (i1 < g.n[1]) nbs += to_d(x[f + s1]);
  if (g.dim == 3) {
    if (i2 > 0) nbs += to_d(x[f - s2]);
    if (i2 < g.n[2]) nbs += to_d(x[f + s2]);
  }
  y[f] = D * to_d(x[f]) - A.op.inv_h2 * nbs;
}

// y = A x in FP32 (helm_apply with HELM_F32)
__global__ void __launch_bounds__(256) k_l1_apply32(L1<float> A, const cf* __restrict__ x,
                                                    cf* __restrict__ y) {
  const Geom& g = A.op.g;
  long long nb = (g.tot + 255) / 256;
  long long f = xcd_block(nb) * 256 + threadIdx.x;
  if (f >= g.tot) return;
  int i0, i1, i2;
  decode(g, f, i0, i1, i2);
  cf D = A.diag(f, i0, i1, i2);
  cf nbs = mk(0.f, 0.f);
  long long s1 = g.N[0], s2 = (long long)g.N[0] * g.N[1];
  if (i0 > 0) nbs += x[f - 1];
  if (i0 < g.n[0]) nbs += x[f + 1];
  if (i1 > 0) nbs += x[f - s1];
  if (i1 < g.n[1]) nbs += x[f + s1];
  if (g.dim == 3) {
    if (i2 > 0) nbs += x[f - s2];
    if (i2 < g.n[2]) nbs += x[f + s2];
  }
  y[f] = D * x[f] - (float)A.op.inv_h2 * nbs;
}

template <typename R, int XIN>
__device__ __forceinline__ typename cplx<R>::type xin_l2(const L2<R>& A, const typename cplx<R>::type* __restrict__ x,
                                                        const typename cplx<R>::type* __restrict__ b, R w,
                                                        const Geom& gc, const typename cplx<R>::type* __restrict__ e,
                                                        long long f, int i0, int i1, int i2) {
  typedef typename cplx<R>::type C;
  C v = mk((R)0, (R)0);
  if (XIN & XIN_X) v += x[f];
  if (XIN & XIN_Z) v += w * cdiv(b[f], A.get(A.center(), f));
  if (XIN & XIN_E) v += prolong_at(gc, e, i0, i1, i2, A.g.dim);
  return v;
}

template <typename R, int XIN>
__device__ __forceinline__ void apply_l2(const L2<R>& A, const typename cplx<R>::type* __restrict__ x,
                                         const typename cplx<R>::type* __restrict__ b, R w_in, const Geom& gc,
                                         const typename cplx<R>::type* __restrict__ e, long long f, int i0,
                                         int i1, int i2, typename cplx<R>::type& Ax,
                                         typename cplx<R>::type& xc, typename cplx<R>::type& D) {
  typedef typename cplx<R>::type C;
  const Geom& g = A.g;
  Ax = mk((R)0, (R)0);
  int r2 = g.dim == 3 ? 1 : 0;
  for (int d2 = -r2; d2 <= r2; ++d2) {
    int j2 = i2 + d2;
    if (j2 < 0 || j2 > g.n[2]) continue;
    for (int d1 = -1; d1 <= 1; ++d1) {
      int j1 = i1 + d1;
      if (j1 < 0 || j1 > g.n[1]) continue;
      for (int d0 = -1; d0 <= 1; ++d0) {
        int j0 = i0 + d0;
        if (j0 < 0 || j0 > g.n[0]) continue;
        int k = (d0 + 1) + 3 * (d1 + 1) + (g.dim == 3 ? 9 * (d2 + 1) : 0);
        long long j = j0 + (long long)g.N[0] * (j1 + (long long)g.N[1] * j2);
        C xj = xin_l2<R, XIN>(A, x, b, w_in, gc, e, j, j0, j1, j2);
        if (k == A.center()) xc = xj;
        Ax += A.get(k, f) * xj;
      }
    }
  }
  D = A.get(A.center(), f);
}

template <typename R, int XIN>
__global__ void __launch_bounds__(256) k_l2_sweep(L2<R> A, const typename cplx<R>::type* __restrict__ x,
                                                  const typename cplx<R>::type* __restrict__ b, R w_in, Geom gc,
                                                  const typename cplx<R>::type* __restrict__ e, R w,
                                                  typename cplx<R>::type* __restrict__ out) {
  typedef typename cplx<R>::type C;
  const Geom& g = A.g;
  long long nb = (g.tot + 255) / 256;
  long long f = xcd_block(nb) * 256 + threadIdx.x;
  if (f >= g.tot) return;
  int i0, i1, i2;
  decode(g, f, i0, i1, i2);
  C Ax, xc, D;
  apply_l2<R, XIN>(A, x, b, w_in, gc, e, f, i0, i1, i2, Ax, xc, D);
  out[f] = xc + w * cdiv(b[f] - Ax, D);
}

template <typename R, int XIN>
__global__ void __launch_bounds__(256) k_l2_restrict(L2<R> A, const typename cplx<R>::type* __restrict__ x,
                                                     const typename cplx<R>::type* __restrict__ b, R w_in,
                                                     Geom gc, const typename cplx<R>::type* __restrict__ e,
                                                     Geom g3, typename cplx<R>::type* __restrict__ b3) {
  typedef typename cplx<R>::type C;
  const Geom& g = A.g;
  long long nb = (g3.tot + 255) / 256;
  long long I = xcd_block(nb) * 256 + threadIdx.x;
  if (I >= g3.tot) return;
  int I0, I1, I2;
  decode(g3, I, I0, I1, I2);
  C acc = mk((R)0, (R)0);
  int r2 = g.dim == 3 ? 1 : 0;
  for (int o2 = -r2; o2 <= r2; ++o2) {
    int f2 = 2 * I2 + o2;
    if (f2 < 0 || f2 > g.n[2]) continue;
    R w2 = (g.dim == 3) ? (o2 == 0 ? (R)0.5 : (R)0.25) : (R)1;
    for (int o1 = -1; o1 <= 1; ++o1) {
      int f1 = 2 * I1 + o1;
      if (f1 < 0 || f1 > g.n[1]) continue;
      R w1 = o1 == 0 ? (R)0.5 : (R)0.25;
      for (int o0 = -1; o0 <= 1; ++o0) {
        int f0 = 2 * I0 + o0;
        if (f0 < 0 || f0 > g.n[0]) continue;
        R w0 = o0 == 0 ? (R)0.5 : (R)0.25;
        long long f = f0 + (long long)g.N[0] * (f1 + (long long)g.N[1] * f2);
        C Ax, xc, D;
        apply_l2<R, XIN>(A, x, b, w_in, gc, e, f, f0, f1, f2, Ax, xc, D);
        acc += (w0 * w1 * w2) * (b[f] - Ax);
      }
    }
  }
  b3[I] = acc;
}

// ------------------------------- launchers ---------------------------------
static inline unsigned grid_for(long long n) { return (unsigned)((n + 255) / 256); }
static inline unsigned grid_xcd(long long n) {
  long long nb = (n + 255) / 256;
  long long per = (nb + 7) / 8;
  return (unsigned)(per * 8);
}

template <typename R, typename CB, typename CO>
void l1_sweep(const L1<R>& A, int xin, const typename cplx<R>::type* x, const CB* b, R w_in, const Geom& gc,
              const typename cplx<R>::type* e, R w, CO* out, hipStream_t s) {
  dim3 grid(grid_xcd(A.op.g.tot)), blk(256);
#define L1S(F) hipLaunchKernelGGL((k_l1_sweep<R, CB, CO, F>), grid, blk, 0, s, A, x, b, w_in, gc, e, w, out)
  switch (xin) {
    case 0: L1S(0); break;
    case XIN_X: L1S(XIN_X); break;
    case XIN_Z: L1S(XIN_Z); break;
    case XIN_E: L1S(XIN_E); break;
    case XIN_X | XIN_E: L1S(XIN_X | XIN_E); break;
    case XIN_Z | XIN_E: L1S(XIN_Z | XIN_E); break;
    default: break;
  }
#undef L1S
}

template <typename R, typename CB>
void l1_restrict(const L1<R>& A, int xin, const typename cplx<R>::type* x, const CB* b, R w_in, const Geom& gc,
                 const typename cplx<R>::type* e, const Geom& g2, typename cplx<R>::type* b2, hipStream_t s) {
  dim3 grid(grid_xcd(g2.tot)), blk(256);
#define L1R(F) hipLaunchKernelGGL((k_l1_restrict<R, CB, F>), grid, blk, 0, s, A, x, b, w_in, gc, e, g2, b2)
  switch (xin) {
    case 0: L1R(0); break;
    case XIN_X: L1R(XIN_X); break;
    case XIN_Z: L1R(XIN_Z); break;
    default: break;
  }
#undef L1R
}

template <typename R>
void l2_sweep(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b, R w_in,
              const Geom& gc, const typename cplx<R>::type* e, R w, typename cplx<R>::type* out, hipStream_t s) {
  dim3 grid(grid_xcd(A.g.tot)), blk(256);
#define L2S(F) hipLaunchKernelGGL((k_l2_sweep<R, F>), grid, blk, 0, s, A, x, b, w_in, gc, e, w, out)
  switch (xin) {
    case 0: L2S(0); break;
    case XIN_X: L2S(XIN_X); break;
    case XIN_Z: L2S(XIN_Z); break;
    case XIN_E: L2S(XIN_E); break;
    case XIN_X | XIN_E: L2S(XIN_X | XIN_E); break;
    case XIN_Z | XIN_E: L2S(XIN_Z | XIN_E); break;
    default: break;
  }
#undef L2S
}

template <typename R>
void l2_restrict(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b,
                 R w_in, const Geom& gc, const typename cplx<R>::type* e, const Geom& g3,
                 typename cplx<R>::type* b3, hipStream_t s) {
  dim3 grid(grid_xcd(g3.tot)), blk(256);
#define L2R(F) hipLaunchKernelGGL((k_l2_restrict<R, F>), grid, blk, 0, s, A, x, b, w_in, gc, e, g3, b3)
  switch (xin) {
    case 0: L2R(0); break;
    case XIN_X: L2R(XIN_X); break;
    case XIN_Z: L2R(XIN_Z); break;
    default: break;
  }
#undef L2R
}

void l1_apply64(const L1<double>& A, const void* x, int x_is_f32, cd* y, hipStream_t s) {
  dim3 grid(grid_xcd(A.op.g.tot)), blk(256);
  if (x_is_f32)
    hipLaunchKernelGGL((k_l1_apply64<cf>), grid, blk, 0, s, A, (const cf*)x, y);
  else
    hipLaunchKernelGGL((k_l1_apply64<cd>), grid, blk, 0, s, A, (const cd*)x, y);
}

void l1_apply32(const L1<float>& A, const cf* x, cf* y, hipStream_t s) {
  dim3 grid(grid_xcd(A.op.g.tot)), blk(256);
  hipLaunchKernelGGL(k_l1_apply32, grid, blk, 0, s, A, x, y);
}

// explicit instantiations used by the cycle driver
template void l1_sweep<float, cd, cf>(const L1<float>&, int, const cf*, const cd*, float,
                                               const Geom&, const cf*, float, cf*, hipStream_t);
template void l1_sweep<float, cd, cd>(const L1<float>&, int, const cf*, const cd*, float,
                                                const Geom&, const cf*, float, cd*, hipStream_t);
template void l1_sweep<double, cd, cd>(const L1<double>&, int, const cd*, const cd*, double,
                                                 const Geom&, const cd*, double, cd*, hipStream_t);
template void l1_restrict<float, cd>(const L1<float>&, int, const cf*, const cd*, float,
                                          const Geom&, const cf*, const Geom&, cf*, hipStream_t);
template void l1_restrict<double, cd>(const L1<double>&, int, const cd*, const cd*, double,
                                           const Geom&, const cd*, const Geom&, cd*, hipStream_t);
template void l2_sweep<float>(const L2<float>&, int, const cf*, const cf*, float, const Geom&,
                              const cf*, float, cf*, hipStream_t);
template void l2_sweep<double>(const L2<double>&, int, const cd*, const cd*, double, const Geom&,
                               const cd*, double, cd*, hipStream_t);
template void l2_restrict<float>(const L2<float>&, int, const cf*, const cf*, float, const Geom&,
                                 const cf*, const Geom&, cf*, hipStream_t);
template void l2_restrict<double>(const L2<double>&, int, const cd*, const cd*, double, const Geom&,
                                  const cd*, const Geom&, cd*, hipStream_t);

}  // namespace helm
