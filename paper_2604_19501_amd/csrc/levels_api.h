// Level-1 / level-2 operator descriptors and cycle-kernel launchers (internal).
#pragma once
#include "internal.h"

namespace helm {

// flags of the "virtual" input iterate of a relaxation / restriction kernel:
// x_in = [stored x] + [w D^-1 b] + [P e]
enum : int { XIN_X = 1, XIN_Z = 2, XIN_E = 4 };

// ----------------------------- level 1 -------------------------------------
// complex coefficient c = s * m * (1 - i sigma) and diagonal 2d/h^2 - c
// sigma of the absorbing layer in the arithmetic of the operator: the FP32 cycle evaluates
// it in FP32 (reciprocal widths multiplied, no division, no branch)
template <typename R>
__device__ __forceinline__ R layer_sigma_r(const FineOp& op, int i0, int i1, int i2) {
  if (sizeof(R) == 8) return (R)layer_sigma(op, i0, i1, i2);
  const int ii[3] = {i0, i1, i2};
  float s = 0.f;
  for (int a = 0; a < op.g.dim; ++a) {
    const float tl = (float)max(op.layer[a][0] - ii[a], 0) * op.inv_wf[a][0];
    const float th = (float)max(ii[a] - op.inner_hi[a], 0) * op.inv_wf[a][1];
    s += tl * tl + th * th;
  }
  return (R)((float)op.sigma_max * s);
}

template <typename R>
struct L1 {
  typedef typename cplx<R>::type C;
  FineOp op;
  C s;                 // (1 - i beta) omega^2 (times alpha^2 for a shifted operator)
  const R* m;          // squared slowness
  int conj;            // 1: coefficients of conj(H) (the adjoint, H being complex symmetric)
  const C* dg = nullptr;   // the FP32 cycle: its diagonal precomputed at set-up (of the
                           // operator, not of its conjugate), read instead of m
  int box_sweep = 0, box_restrict = 0;   // box-shape variants of the tiled kernels
  // the coefficient and the diagonal from the node's squared slowness mm = m[f]
  __device__ __forceinline__ C coef_m(R mm, int i0, int i1, int i2) const {
    R sig = layer_sigma_r<R>(op, i0, i1, i2);
    C c = mk(mm, -mm * sig);        // m (1 - i sigma)
    C r = s * c;
    if (conj) r.y = -r.y;
    return r;
  }
  __device__ __forceinline__ C diag_m(R mm, int i0, int i1, int i2) const {
    C c = coef_m(mm, i0, i1, i2);
    return mk((R)(2.0 * op.g.dim * op.inv_h2) - c.x, -c.y);
  }
  __device__ __forceinline__ C coef(long long f, int i0, int i1, int i2) const { return coef_m(m[f], i0, i1, i2); }
  __device__ __forceinline__ C diag(long long f, int i0, int i1, int i2) const { return diag_m(m[f], i0, i1, i2); }
};

// ----------------------------- level 2 -------------------------------------
template <typename R>
struct L2 {
  typedef typename cplx<R>::type C;
  Geom g;
  const C* coef;     // SoA, plane k at coef[k * N]: 3^d planes, or (SYM2) the centre and the
                     // 13 directions after it
  int conj;          // use conj(coef) (adjoint)
  int box_sweep = 0, box_restrict = 0;   // box-shape variants of the tiled kernels
  __device__ __forceinline__ C get(int k, long long i) const {
    C c = coef[(long long)k * g.tot + i];
    if (conj) c.y = -c.y;
    return c;
  }
  // coefficient k of node i of the complex-symmetric 3D operator stored from its centre on:
  // A(i, i + d) = A(i + d, i), so a direction before the centre reads the mirrored one at
  // the neighbour.  Where i + d lies outside the grid the product is with a zero iterate;
  // the index is clamped into the array.
  __device__ __forceinline__ C get_sym3(int k, long long i) const {
    C c;
    if (k >= 13) {
      c = coef[(long long)(k - 13) * g.tot + i];
    } else {
      const long long off = (k % 3 - 1) + (long long)g.N[0] * ((k / 3) % 3 - 1 + (long long)g.N[1] * (k / 9 - 1));
      const long long j = min(max(i + off, 0LL), g.tot - 1);
      c = coef[(long long)(13 - k) * g.tot + j];
    }
    if (conj) c.y = -c.y;
    return c;
  }
  __device__ __forceinline__ int center() const { return g.dim == 2 ? 4 : 13; }
};


// nrhs right-hand sides at once: the vectors of right-hand side r follow those of r - 1
// at one level size (x, b, out at the operator's level, e at the coarse level)
template <typename R, typename CB, typename CO>
void l1_sweep(const L1<R>& A, int xin, const typename cplx<R>::type* x, const CB* b, R w_in, const Geom& gc,
              const typename cplx<R>::type* e, R w, CO* out, int nrhs, hipStream_t s);
template <typename R, typename CB>
void l1_restrict(const L1<R>& A, int xin, const typename cplx<R>::type* x, const CB* b, R w_in, const Geom& gc,
                 const typename cplx<R>::type* e, const Geom& g2, typename cplx<R>::type* b2, int nrhs,
                 hipStream_t s);
template <typename R>
void l2_sweep(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b, R w_in,
              const Geom& gc, const typename cplx<R>::type* e, R w, typename cplx<R>::type* out, int nrhs,
              hipStream_t s);
template <typename R>
void l2_restrict(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b,
                 R w_in, const Geom& gc, const typename cplx<R>::type* e, const Geom& g3,
                 typename cplx<R>::type* b3, int nrhs, hipStream_t s);
// 2D, between the two level-2 visits of a W-cycle with one pre- and one post-sweep: the
// post-sweep of the first visit (xin = XIN_Z | XIN_E, e the coarse correction on gc), the
// pre-sweep of the next (xb receives its iterate) and that visit's residual, restricted into
// b3 on gc, in one launch
template <typename R>
void l2_chain(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b, R w_in,
              const Geom& gc, const typename cplx<R>::type* e, R w, typename cplx<R>::type* xb,
              typename cplx<R>::type* b3, int nrhs, hipStream_t s);
// 2D, the end of a cycle with one post-sweep on each level: the last level-2 post-sweep
// (from x2 + P e3, e3 on g3) and the level-1 post-sweep (from the virtual first sweep
// w1 D1^-1 b1 plus the prolongated level-2 result) into out, in one launch; the level-2
// iterate is not written
template <typename R, typename CO>
void cycle_tail(const L1<R>& A1, const cd* b1, R w1, const L2<R>& A2, const typename cplx<R>::type* x2,
                const typename cplx<R>::type* b2, R w2, const Geom& g3, const typename cplx<R>::type* e3, CO* out,
                int nrhs, hipStream_t s);
void l1_apply64(const L1<double>& A, const void* x, int x_is_f32, cd* y, hipStream_t s);
// dg[f] = the diagonal of A at every node (set-up of the FP32 cycle's level-1 operator)
void l1_diag32(const L1<float>& A, cf* dg, hipStream_t s);
void l1_apply32(const L1<float>& A, const cf* x, cf* y, hipStream_t s);

}  // namespace helm
