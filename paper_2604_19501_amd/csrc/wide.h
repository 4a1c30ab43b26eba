// The paper's compact fourth-order stack (internal): kernels of its three-level cycle and
// of its Galerkin operators.
//
//   fine     H = L_h - M_h diag(c), c = s m (1 - i sigma)                  (eqs. 3.1, 3.2)
//            L_h: (1/6h^2)[-1 -4 -1; -4 20 -4; -1 -4 -1] (2D),
//                 (1/6h^2)(24 centre, -2 faces, -1 edges) (3D);
//            M_h: centre 8/12 (2D) or 6/12 (3D), faces 1/12; zero values outside the grid
//   transfer R = tensor product of [1 4 6 4 1]/16 ("cubic", eq. 3.3) or of [1 2 1]/4;
//            P = 2^d R'^T of the interpolating restriction R' (cubic in every case, so
//            "level-dependent", eq. 3.4, only changes the restriction from level 2 to 3)
//   level 2  A2 = R1 H_beta^{alpha2} P1: radius 2 (25 / 125 points)
//   level 3  A3 = R2 (R1 H_beta^alpha P1) P2: radius 3 (49 points, cubic 2D) or 2
//            (level-dependent transfers: 25 / 125 points)
//
// Stored operators are coefficient planes: entry A(i, i + d), |d_a| <= r, at
// coef[k N + i] with k = sum_a (d_a + r) (2r + 1)^a.
#pragma once
#include "levels_api.h"

namespace helm {

// 1-D weights of a restriction: offsets -a..a, w[o + a]
struct Transfer1D {
  int a;
  double w[5];
};
inline Transfer1D transfer_cubic() { return Transfer1D{2, {1 / 16., 4 / 16., 6 / 16., 4 / 16., 1 / 16.}}; }
inline Transfer1D transfer_fw() { return Transfer1D{1, {0.25, 0.5, 0.25, 0.0, 0.0}}; }

// the fine compact operator with coefficient scalar s in precision R; conj is not
// supported (the operator is not complex symmetric)
template <typename R>
struct WFine {
  typedef typename cplx<R>::type C;
  FineOp op;
  C s;                // alpha^2 (1 - i beta) omega^2
  const R* m;         // squared slowness
};

// ---- set-up (FP64) ----
// out (planes of radius rc on gc) = Rt-restriction of H_s (compact, fine grid op.g)
// interpolated by Pt (P = 2^d Pt^T per axis)
void wgal_fine(const FineOp& op, cd s, const double* m, const Geom& gc, const Transfer1D& Rt,
               const Transfer1D& Pt, int rc, cd* out, hipStream_t st);
// out = Rt A Pt for A given as planes of radius rin on g
void wgal_coarse(const Geom& g, const cd* A, int rin, const Geom& gc, const Transfer1D& Rt, const Transfer1D& Pt,
                 int rc, cd* out, hipStream_t st);

// ---- cycle kernels (nr right-hand sides in grid y, vectors N apart) ----
enum : int { WM_RES = 0, WM_JAC = 1, WM_APPLY = 2 };
// level 1: WM_RES out = b - H x; WM_JAC out = x + w (b - H x) / diag(H); WM_APPLY out = H x.
// xz: x is zero (not read)
template <typename R, typename CB, typename CO>
void w1_step(const WFine<R>& A, int mode, int xz, const typename cplx<R>::type* x, const CB* b, R w, CO* out,
             int nr, hipStream_t st);
// level 2 (planes of radius r = 2, the compact stack's level-2 operator, in precision R): the
// same three modes
template <typename R>
void w2_step(const Geom& g, const typename cplx<R>::type* coef, int r, int mode, int xz,
             const typename cplx<R>::type* x, const typename cplx<R>::type* b, R w, typename cplx<R>::type* out,
             int nr, hipStream_t st);
// out(I) = sum_i R(I, i) v(i) from grid gf onto gc (summed in v's precision, stored in out's)
template <typename CI, typename CO>
void w_restrict(const Geom& gf, const CI* v, const Geom& gc, const Transfer1D& Rt, CO* out, int nr, hipStream_t st);
// x(i) = [x(i)] + sum_J P(i, J) e(J), P = 2^d Pt^T, from gc onto gf (add: keep x); summed in
// x's precision
template <typename CE, typename C>
void w_prolong(const Geom& gc, const CE* e, const Geom& gf, const Transfer1D& Pt, int add, C* x, int nr,
               hipStream_t st);
// out = in, converted to out's precision (n entries)
template <typename CI, typename CO>
void w_copy(const CI* in, CO* out, long long n, hipStream_t st);

// the absorbing layer's squared depth term on axis A at index i (the summand of
// layer_sigma for that axis), in the arithmetic of R
template <typename R, int A>
__device__ __forceinline__ R layer_t2(const FineOp& op, int i) {
  const R wl = sizeof(R) == 4 ? (R)op.inv_wf[A][0] : (R)op.inv_w[A][0];
  const R wh = sizeof(R) == 4 ? (R)op.inv_wf[A][1] : (R)op.inv_w[A][1];
  const R tl = (R)max(op.layer[A][0] - i, 0) * wl;
  const R th = (R)max(i - op.inner_hi[A], 0) * wh;
  return tl * tl + th * th;
}

// Row f (node i0, i1, i2) of the fine compact operator with coefficient scalar s, applied
// to x (any precision) in the arithmetic of R; dg receives the diagonal L_ff - M_ff c_f.
// xz: x is zero (only dg is computed).  Neighbours outside the grid are read at f and
// weighted 0, so that every load is issued unconditionally.
template <int DIM, typename R, typename CX>
__device__ __forceinline__ typename cplx<R>::type wide_row(const FineOp& op, typename cplx<R>::type s,
                                                           const R* __restrict__ m, const CX* __restrict__ x,
                                                           long long f, int i0, int i1, int i2, bool xz,
                                                           typename cplx<R>::type& dg) {
  typedef typename cplx<R>::type C;
  const Geom& g = op.g;
  const R ih = (R)(op.inv_h2 / 6.0);
  const long long s1 = g.N[0], s2 = (long long)g.N[0] * g.N[1];
  const R lc = DIM == 3 ? (R)24 : (R)20;                       // L: centre (x 1/6h^2)
  const R lf = DIM == 3 ? (R)-2 : (R)-4;                       // L: faces
  const R mc = DIM == 3 ? (R)(6.0 / 12.0) : (R)(8.0 / 12.0);   // M: centre
  const R mf = (R)(1.0 / 12.0);                                // M: faces
  // sigma at the node and its face neighbours from per-axis terms (a face neighbour differs
  // in one axis), summed in axis order as layer_sigma does
  const R smax = (R)op.sigma_max;
  R tc[3], tm[3], tp[3];
  tc[0] = layer_t2<R, 0>(op, i0);
  tm[0] = layer_t2<R, 0>(op, i0 - 1);
  tp[0] = layer_t2<R, 0>(op, i0 + 1);
  tc[1] = layer_t2<R, 1>(op, i1);
  tm[1] = layer_t2<R, 1>(op, i1 - 1);
  tp[1] = layer_t2<R, 1>(op, i1 + 1);
  tc[2] = tm[2] = tp[2] = (R)0;
  if (DIM == 3) {
    tc[2] = layer_t2<R, 2>(op, i2);
    tm[2] = layer_t2<R, 2>(op, i2 - 1);
    tp[2] = layer_t2<R, 2>(op, i2 + 1);
  }
  auto sig = [&](int ax, int dir) -> R {     // ax < 0: the node itself
    R t = (R)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) t += a != ax ? tc[a] : (dir < 0 ? tm[a] : tp[a]);
    return smax * t;
  };
  const R mm0 = m[f];
  const C c0 = s * mk(mm0, -mm0 * sig(-1, 0));
  dg = mk(lc * ih - mc * c0.x, -mc * c0.y);
  C acc = mk((R)0, (R)0);
  if (xz) return acc;
  acc = dg * conv<C>::from(x[f]);
#pragma unroll
  for (int d2 = (DIM == 3 ? -1 : 0); d2 <= (DIM == 3 ? 1 : 0); ++d2)
#pragma unroll
    for (int d1 = -1; d1 <= 1; ++d1)
#pragma unroll
      for (int d0 = -1; d0 <= 1; ++d0) {
        const int nz = (d0 != 0) + (d1 != 0) + (d2 != 0);
        if (nz == 0 || nz == 3) continue;          // the centre (above); 3D corners: zero
        const int a0 = i0 + d0, a1 = i1 + d1, a2 = i2 + d2;
        const bool in = a0 >= 0 && a0 <= g.n[0] && a1 >= 0 && a1 <= g.n[1] &&
                        (DIM == 2 || (a2 >= 0 && a2 <= g.n[2]));
        const long long j = in ? f + d0 + d1 * s1 + d2 * s2 : f;
        const C xv = conv<C>::from(x[j]);
        const R on = in ? (R)1 : (R)0;
        if (nz == 1) {                              // face: L and M entries
          const R mj = m[j];
          const int ax = d0 != 0 ? 0 : d1 != 0 ? 1 : 2, dir = d0 + d1 + d2;
          const C cj = s * mk(mj, -mj * sig(ax, dir));
          const C a = mk(lf * ih - mf * cj.x, -mf * cj.y);
          acc += on * (a * xv);
        } else {                                    // 2D corner / 3D edge: L only (-1)
          acc -= (on * ih) * xv;
        }
      }
  return acc;
}

}  // namespace helm
