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
#include <type_traits>

#include "levels_api.h"

namespace helm {



// a / d for the Jacobi updates: in the FP32 cycle one hardware reciprocal of |d|^2 (about
// 1 ulp) replaces two IEEE divisions; FP64 keeps the exact quotient
__device__ __forceinline__ cf jdiv(cf a, cf d) {
  const float r = __builtin_amdgcn_rcpf(d.x * d.x + d.y * d.y);
  return mk((a.x * d.x + a.y * d.y) * r, (a.y * d.x - a.x * d.y) * r);
}
__device__ __forceinline__ cd jdiv(cd a, cd d) { return cdiv(a, d); }

// contiguous-slab block order: hardware dispatches block b to XCD b % 8
__device__ __forceinline__ long long xcd_block(long long nblocks) {
  long long b = blockIdx.x;
  long long per = (nblocks + 7) / 8;
  long long xcd = b % 8, k = b / 8;
  long long lb = xcd * per + k;
  return lb;   // may exceed nblocks - 1: caller bounds-checks
}

__device__ __forceinline__ void decode(const Geom& g, long long f, int& i0, int& i1, int& i2) {
  node_coords(g, f, i0, i1, i2);
}

__device__ __forceinline__ bool inside(const Geom& g, int i0, int i1, int i2) {
  return i0 >= 0 && i0 <= g.n[0] && i1 >= 0 && i1 <= g.n[1] && i2 >= 0 && i2 <= g.n[2];
}
// node index in 32 bits (grids are validated to hold fewer than 2^31 nodes); the
// right-hand side offsets are applied to the base pointers
__device__ __forceinline__ int flat(const Geom& g, int i0, int i1, int i2) {
  return i0 + g.N[0] * (i1 + g.N[1] * i2);
}

// ----------------------------------------------------------------------------
// Tiled kernels.  A block owns a box of output nodes.  It stages in LDS
//   * the coarse correction e on the box's coarse footprint (sweeps with XIN_E),
//   * the virtual input iterate x_in on the box plus a one-node halo,
//   * for restrictions, the residual b - A x_in on the (2c+1)^d fine footprint,
// so every x_in and every residual is evaluated once per node (plus the halo)
// and every global array is read with x-consecutive lanes.  Nodes outside the
// grid are stored as zero, which is the operator's boundary condition (zero
// values one node outside); the stored coarse coefficients that point outside
// are zero as well.
//
// Box shapes (threads = 256), chosen per context (L1/L2::box_sweep, box_restrict; the
// autotuner picks them), variant 0 the default:
//   sweeps       2D 32 x 16, 64 x 8, 64 x 16, 32 x 32
//                3D 32 x 8 x 4, 32 x 8 x 8, 64 x 8 x 4, 32 x 16 x 4
//   restrictions 2D 16 x 8, 32 x 8, 16 x 16 coarse
//                3D 8 x 4 x 4, 16 x 4 x 4, 8 x 8 x 4 coarse
//   and, 3D FP32 only, z-marching tiles (below): sweeps 4 and 5, restrictions 3 and 4
//   (in 2D these variants run variant 0).
// The FP64 cycle keeps variant 0 in 3D (the others exceed the block's LDS).
template <int DIM, int V> struct SBox {
  static constexpr int x = DIM == 2 ? (V == 0 || V == 3 ? 32 : 64) : (V == 2 ? 64 : 32);
  static constexpr int y = DIM == 2 ? (V == 0 ? 16 : V == 1 ? 8 : V == 2 ? 16 : 32) : (V == 3 ? 16 : 8);
  static constexpr int z = DIM == 2 ? 1 : (V == 1 ? 8 : 4);
};
template <int DIM, int V> struct RBox {
  static constexpr int x = DIM == 2 ? (V == 1 ? 32 : 16) : (V == 1 ? 16 : 8);
  static constexpr int y = DIM == 2 ? (V == 2 ? 16 : 8) : (V == 2 ? 8 : 4);
  static constexpr int z = DIM == 2 ? 1 : 4;
};
constexpr int N_SBOX = 6, N_RBOX = 5;
// z-marching tiles: an xy tile of output nodes over z consecutive planes
//   sweeps       30 x 14 nodes, 16 (variant 4) or 4 (variant 5) planes
//   restrictions 14 x 6 coarse nodes, 8 (variant 3) or 4 (variant 4) coarse planes
// (the staged planes, 32 x 16 and 31 x 15 nodes, take two wavefront passes of 256 threads)
template <int V> struct ZSBox {
  static constexpr int x = 30, y = 14, z = V == 4 ? 16 : 4;
};
template <int V> struct ZRBox {
  static constexpr int x = 14, y = 6, z = V == 3 ? 8 : 4;
};

// level-1 operator H_s with x from LDS (centre index k, strides sy, sz).  The FP32 cycle
// reads its diagonal from the array precomputed at set-up (one 8-byte load per node instead
// of the squared slowness, the layer profile and the complex coefficient: the level-1
// kernels are bound by instruction issue as much as by memory); FP64 evaluates it from m.
template <int DIM, typename R>
struct Op1 {
  typedef R Real;
  typedef typename cplx<R>::type C;
  static constexpr bool DG = sizeof(R) == 4;
  L1<R> A;
  __host__ __device__ __forceinline__ const Geom& geom() const { return A.op.g; }
  __device__ __forceinline__ C dg_at(long long f) const {
    C d = A.dg[f];
    if (A.conj) d.y = -d.y;
    return d;
  }
  __device__ __forceinline__ C diag(long long f, int i0, int i1, int i2) const {
    if constexpr (DG) return dg_at(f);
    else return A.diag(f, i0, i1, i2);
  }
  // the diagonal in two steps, so that the load can be issued early: aux(f), then diag_aux
  typedef typename std::conditional<DG, C, R>::type Aux;
  __device__ __forceinline__ Aux aux(long long f) const {
    if constexpr (DG) return dg_at(f);
    else return A.m[f];
  }
  __device__ __forceinline__ C diag_aux(Aux a, int i0, int i1, int i2) const {
    if constexpr (DG) return a;
    else return A.diag_m(a, i0, i1, i2);
  }
  __device__ __forceinline__ C ax(const C* xs, int k, int sy, int sz, long long, C D) const {
    C nb = (xs[k - 1] + xs[k + 1]) + (xs[k - sy] + xs[k + sy]);
    if (DIM == 3) nb += xs[k - sz] + xs[k + sz];
    return D * xs[k] - (R)A.op.inv_h2 * nb;
  }
  // 3D, the planes below / at / above the node staged apart (z-marching tiles); the same
  // sums in the same order as ax
  __device__ __forceinline__ C ax3(const C* xm, const C* x0, const C* xp, int k, int sy, long long, C D) const {
    C nb = (x0[k - 1] + x0[k + 1]) + (x0[k - sy] + x0[k + sy]);
    nb += xm[k] + xp[k];
    return D * x0[k] - (R)A.op.inv_h2 * nb;
  }
};

// level-2 Galerkin operator (3^d coefficients per node; the 3D FP32 cycle stores the
// complex-symmetric operator from its centre on)
template <int DIM, typename R>
struct Op2 {
  typedef R Real;
  typedef typename cplx<R>::type C;
  static constexpr bool SYM = DIM == 3 && sizeof(R) == 4;
  L2<R> A;
  __host__ __device__ __forceinline__ const Geom& geom() const { return A.g; }
  __device__ __forceinline__ C coef_at(int k, long long f) const { return SYM ? A.get_sym3(k, f) : A.get(k, f); }
  __device__ __forceinline__ C diag(long long f, int, int, int) const { return coef_at(DIM == 2 ? 4 : 13, f); }
  typedef C Aux;
  __device__ __forceinline__ Aux aux(long long f) const { return coef_at(DIM == 2 ? 4 : 13, f); }
  __device__ __forceinline__ C diag_aux(Aux d, int, int, int) const { return d; }
  __device__ __forceinline__ C ax(const C* xs, int k, int sy, int sz, long long f, C D) const {
    C acc = D * xs[k];
#pragma unroll
    for (int d2 = (DIM == 3 ? -1 : 0); d2 <= (DIM == 3 ? 1 : 0); ++d2)
#pragma unroll
      for (int d1 = -1; d1 <= 1; ++d1)
#pragma unroll
        for (int d0 = -1; d0 <= 1; ++d0) {
          if (d0 == 0 && d1 == 0 && d2 == 0) continue;
          const int kk = (d0 + 1) + 3 * (d1 + 1) + (DIM == 3 ? 9 * (d2 + 1) : 0);
          acc += coef_at(kk, f) * xs[k + d0 + sy * d1 + sz * d2];
        }
    return acc;
  }
  __device__ __forceinline__ C ax3(const C* xm, const C* x0, const C* xp, int k, int sy, long long f, C D) const {
    C acc = D * x0[k];
#pragma unroll
    for (int d2 = -1; d2 <= 1; ++d2)
#pragma unroll
      for (int d1 = -1; d1 <= 1; ++d1)
#pragma unroll
        for (int d0 = -1; d0 <= 1; ++d0) {
          if (d0 == 0 && d1 == 0 && d2 == 0) continue;
          const int kk = (d0 + 1) + 3 * (d1 + 1) + 9 * (d2 + 1);
          const C* pl = d2 < 0 ? xm : d2 > 0 ? xp : x0;
          acc += coef_at(kk, f) * pl[k + d0 + sy * d1];
        }
    return acc;
  }
};

// d-linear interpolation of the staged coarse vector at fine node (i0,i1,i2); a
// coordinate on a coarse node reads the same value twice with weight 1/2 each,
// which is exact
template <int DIM, typename C>
__device__ __forceinline__ C prolong_lds(const C* es, int ex, int ey, int c0, int c1, int c2, int i0, int i1,
                                         int i2) {
  typedef decltype(es[0].x) R;
  const int l0 = (i0 >> 1) - c0, h0 = ((i0 + 1) >> 1) - c0;
  const int l1 = (i1 >> 1) - c1, h1 = ((i1 + 1) >> 1) - c1;
  if (DIM == 2) {
    C v = (es[l0 + ex * l1] + es[h0 + ex * l1]) + (es[l0 + ex * h1] + es[h0 + ex * h1]);
    return (R)0.25 * v;
  } else {
    const int l2 = (i2 >> 1) - c2, h2 = ((i2 + 1) >> 1) - c2;
    const int pl = ex * ey * l2, ph = ex * ey * h2;
    C v = ((es[l0 + ex * l1 + pl] + es[h0 + ex * l1 + pl]) + (es[l0 + ex * h1 + pl] + es[h0 + ex * h1 + pl])) +
          ((es[l0 + ex * l1 + ph] + es[h0 + ex * l1 + ph]) + (es[l0 + ex * h1 + ph] + es[h0 + ex * h1 + ph]));
    return (R)0.125 * v;
  }
}

struct TileGrid {
  int nt[3];
  int ntiles;
};

// the block's tile, in 32-bit arithmetic on values uniform over the block
__device__ __forceinline__ bool tile_origin(const TileGrid& tg, int bx, int by, int bz, int& o0, int& o1,
                                           int& o2) {
  const int b = blockIdx.x, per = (tg.ntiles + 7) >> 3;
  const int t = __builtin_amdgcn_readfirstlane((b & 7) * per + (b >> 3));
  if (t >= tg.ntiles) return false;
  const int q = t / tg.nt[0];
  o0 = (t - q * tg.nt[0]) * bx;
  const int q2 = q / tg.nt[1];
  o1 = (q - q2 * tg.nt[1]) * by;
  o2 = q2 * bz;
  return true;
}

// clamp a node to the grid (loads then stay in bounds and are issued unconditionally;
// the caller zeroes what lies outside)
__device__ __forceinline__ void clamp_node(const Geom& g, int& i0, int& i1, int& i2) {
  i0 = min(max(i0, 0), g.n[0]);
  i1 = min(max(i1, 0), g.n[1]);
  i2 = min(max(i2, 0), g.n[2]);
}

// stage x_in on the box [s0, s0+SX) x [s1, s1+SY) x [s2, s2+SZ).  2D: the loads of all of
// a thread's nodes are issued into registers first, then the values are formed and stored,
// so the block waits for memory once.  3D (8 or 9 passes): groups of 4 unrolled passes
// leave the scheduling to the compiler, which keeps the registers at about 70 and 7
// wavefronts per SIMD; explicit register staging of every pass measured slower there
// (about 100 registers, 4 wavefronts per SIMD).  Indices are clamped so every load is
// issued.
template <int DIM, int XIN, int SX, int SY, int SZ, class Op, typename C, typename CB, typename R>
__device__ __forceinline__ void stage_xin(const Op& op, const C* __restrict__ x, const CB* __restrict__ b, R w_in,
                                          const C* es, int ex, int ey, int c0, int c1, int c2, int s0, int s1,
                                          int s2, C* xs) {
  const Geom& g = op.geom();
  constexpr int tot = SX * SY * SZ, NIT = (tot + 255) / 256;
  if constexpr (DIM == 2) {
    C rx[(XIN & XIN_X) ? NIT : 1];
    CB rb[(XIN & XIN_Z) ? NIT : 1];
    typename Op::Aux ra[(XIN & XIN_Z) ? NIT : 1];
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int k = min((int)threadIdx.x + 256 * u, tot - 1);
      const int a = k % SX, q = k / SX;
      int j0 = s0 + a, j1 = s1 + q % SY, j2 = s2 + q / SY;
      clamp_node(g, j0, j1, j2);
      const int f = flat(g, j0, j1, j2);
      if (XIN & XIN_X) rx[(XIN & XIN_X) ? u : 0] = x[f];
      if (XIN & XIN_Z) {
        rb[(XIN & XIN_Z) ? u : 0] = b[f];
        ra[(XIN & XIN_Z) ? u : 0] = op.aux(f);
      }
    }
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int k = min((int)threadIdx.x + 256 * u, tot - 1);
      const int a = k % SX, q = k / SX;
      const int i0 = s0 + a, i1 = s1 + q % SY, i2 = s2 + q / SY;
      int j0 = i0, j1 = i1, j2 = i2;
      clamp_node(g, j0, j1, j2);
      C v = mk((R)0, (R)0);
      if (XIN & XIN_X) v += rx[(XIN & XIN_X) ? u : 0];
      if (XIN & XIN_Z)
        v += w_in * jdiv(conv<C>::from(rb[(XIN & XIN_Z) ? u : 0]), op.diag_aux(ra[(XIN & XIN_Z) ? u : 0], j0, j1, j2));
      if (XIN & XIN_E) v += prolong_lds<DIM>(es, ex, ey, c0, c1, c2, j0, j1, j2);
      if (!inside(g, i0, i1, i2)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * u < tot) xs[k] = v;
    }
  } else {
    for (int i4 = 0; i4 < NIT; i4 += 4)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int it = i4 + u;
      if (NIT % 4 != 0 && it >= NIT) break;
      const int k = min((int)threadIdx.x + 256 * it, tot - 1);
      const int a = k % SX, q = k / SX;
      const int i0 = s0 + a, i1 = s1 + q % SY, i2 = s2 + q / SY;
      int j0 = i0, j1 = i1, j2 = i2;
      clamp_node(g, j0, j1, j2);
      const int f = flat(g, j0, j1, j2);
      C v = mk((R)0, (R)0);
      if (XIN & XIN_X) v += x[f];
      if (XIN & XIN_Z) v += w_in * jdiv(conv<C>::from(b[f]), op.diag(f, j0, j1, j2));
      if (XIN & XIN_E) v += prolong_lds<DIM>(es, ex, ey, c0, c1, c2, j0, j1, j2);
      if (!inside(g, i0, i1, i2)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * it < tot) xs[k] = v;
    }
  }
}

// x_out = x_in + w D^{-1}(b - A x_in) on one box (w = 0: materialise x_in).  The output
// nodes' b and D are loaded before the staging barriers, so their latency overlaps it.
template <int DIM, class Op, typename CB, typename CO, int XIN, int BV>
__global__ void __launch_bounds__(256) k_sweep(Op op, const typename Op::C* __restrict__ x,
                                               const CB* __restrict__ b, typename Op::Real w_in, Geom gc,
                                               const typename Op::C* __restrict__ e,
                                               typename Op::Real w, CO* __restrict__ out, TileGrid tg) {
  typedef typename Op::C C;
  typedef typename Op::Real R;
  constexpr int TX = SBox<DIM, BV>::x, TY = SBox<DIM, BV>::y, TZ = SBox<DIM, BV>::z;
  constexpr int SX = TX + 2, SY = TY + 2, SZ = DIM == 3 ? TZ + 2 : 1;
  constexpr int EX = TX / 2 + 3, EY = TY / 2 + 3, EZ = DIM == 3 ? TZ / 2 + 3 : 1;
  constexpr int NOUT = TX * TY * TZ / 256;
  __shared__ C xs[SX * SY * SZ];
  __shared__ C es[(XIN & XIN_E) ? EX * EY * EZ : 1];
  const Geom& g = op.geom();
  // right-hand side blockIdx.y: its vectors follow each other, one level-size apart
  const long long ry = blockIdx.y;
  if (XIN & XIN_X) x += ry * g.tot;
  b += ry * g.tot;
  if (XIN & XIN_E) e += ry * gc.tot;
  out += ry * g.tot;
  int o0, o1, o2;
  if (!tile_origin(tg, TX, TY, TZ, o0, o1, o2)) return;
  const int s0 = o0 - 1, s1 = o1 - 1, s2 = DIM == 3 ? o2 - 1 : 0;
  const int c0 = s0 >> 1, c1 = s1 >> 1, c2 = s2 >> 1;   // floor: s may be -1
  if (XIN & XIN_E) {
    constexpr int tot = EX * EY * EZ, NIT = (tot + 255) / 256;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int k = min((int)threadIdx.x + 256 * it, tot - 1);
      const int a = k % EX, q = k / EX;
      const int j0 = c0 + a, j1 = c1 + q % EY, j2 = (DIM == 3 ? c2 : 0) + q / EY;
      int l0 = j0, l1 = j1, l2 = j2;
      clamp_node(gc, l0, l1, l2);
      C v = e[flat(gc, l0, l1, l2)];
      if (!inside(gc, j0, j1, j2)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * it < tot) es[k] = v;
    }
  }
  C bo[NOUT], Do[NOUT];
#pragma unroll
  for (int it = 0; it < NOUT; ++it) {
    const int k = (int)threadIdx.x + 256 * it;
    const int a = k % TX, q = k / TX;
    int i0 = o0 + a, i1 = o1 + q % TY, i2 = o2 + q / TY;
    clamp_node(g, i0, i1, i2);
    const int f = flat(g, i0, i1, i2);
    bo[it] = conv<C>::from(b[f]);
    Do[it] = op.diag(f, i0, i1, i2);
  }
  constexpr int STOT = SX * SY * SZ, SIT = (STOT + 255) / 256;
  if ((XIN & XIN_E) && SIT <= 4) {
    // the staged nodes' inputs are loaded before the barrier that publishes e, so one
    // memory round trip serves the block
    typename Op::C rx[SIT];
    CB rb[SIT];
    typename Op::Aux ra[SIT];
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int k = min((int)threadIdx.x + 256 * it, STOT - 1);
      const int a = k % SX, q = k / SX;
      int j0 = s0 + a, j1 = s1 + q % SY, j2 = s2 + q / SY;
      clamp_node(g, j0, j1, j2);
      const int f = flat(g, j0, j1, j2);
      if (XIN & XIN_X) rx[it] = x[f];
      if (XIN & XIN_Z) {
        rb[it] = b[f];
        ra[it] = op.aux(f);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int k = min((int)threadIdx.x + 256 * it, STOT - 1);
      const int a = k % SX, q = k / SX;
      const int i0 = s0 + a, i1 = s1 + q % SY, i2 = s2 + q / SY;
      int j0 = i0, j1 = i1, j2 = i2;
      clamp_node(g, j0, j1, j2);
      C v = prolong_lds<DIM>(es, EX, EY, c0, c1, c2, j0, j1, j2);
      if (XIN & XIN_X) v += rx[it];
      if (XIN & XIN_Z) v += w_in * jdiv(conv<C>::from(rb[it]), op.diag_aux(ra[it], j0, j1, j2));
      if (!inside(g, i0, i1, i2)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * it < STOT) xs[k] = v;
    }
  } else {
    if (XIN & XIN_E) __syncthreads();
    stage_xin<DIM, XIN, SX, SY, SZ>(op, x, b, w_in, es, EX, EY, c0, c1, c2, s0, s1, s2, xs);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NOUT; ++it) {
    const int k = (int)threadIdx.x + 256 * it;
    const int a = k % TX, q = k / TX;
    const int i0 = o0 + a, i1 = o1 + q % TY, i2 = o2 + q / TY;
    if (!inside(g, i0, i1, i2)) continue;
    const int f = flat(g, i0, i1, i2);
    const int kk = (a + 1) + SX * ((q % TY + 1) + SY * (DIM == 3 ? q / TY + 1 : 0));
    const C r = bo[it] - op.ax(xs, kk, SX, SX * SY, f, Do[it]);
    out[f] = conv<CO>::from(xs[kk] + w * jdiv(r, Do[it]));
  }
}

// b_c(I) = sum_f R(I, f) (b - A x_in)(f), full weighting [1 2 1]/4 per axis, one coarse box
template <int DIM, class Op, typename CB, int XIN, int BV>
__global__ void __launch_bounds__(256) k_restrict(Op op, const typename Op::C* __restrict__ x,
                                                  const CB* __restrict__ b, typename Op::Real w_in,
                                                  Geom g2, typename Op::C* __restrict__ b2, TileGrid tg) {
  typedef typename Op::C C;
  typedef typename Op::Real R;
  constexpr int CX = RBox<DIM, BV>::x, CY = RBox<DIM, BV>::y, CZ = RBox<DIM, BV>::z;
  constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1, RZ = DIM == 3 ? 2 * CZ + 1 : 1;
  constexpr int SX = RX + 2, SY = RY + 2, SZ = DIM == 3 ? RZ + 2 : 1;
  constexpr int RT = RX * RY * RZ, NR = (RT + 255) / 256;
  // 3D: the residuals are held in registers until every thread has read the staged
  // iterate, then written over it, which halves the block's LDS (4 blocks per CU
  // instead of 2)
  constexpr bool ALIAS = XIN != 0 && DIM == 3;
  __shared__ C xs[XIN ? SX * SY * SZ : 1];
  __shared__ C rs_own[ALIAS ? 1 : RT];
  C* rs = ALIAS ? xs : rs_own;
  const Geom& g = op.geom();
  const long long ry = blockIdx.y;           // right-hand side
  if (XIN & XIN_X) x += ry * g.tot;
  b += ry * g.tot;
  b2 += ry * g2.tot;
  int O0, O1, O2;
  if (!tile_origin(tg, CX, CY, CZ, O0, O1, O2)) return;
  const int r0 = 2 * O0 - 1, r1 = 2 * O1 - 1, r2 = DIM == 3 ? 2 * O2 - 1 : 0;
  // the residual footprint's b and D, loaded before the staging barrier when it takes at
  // most 4 passes (2D); otherwise in the residual loop
  constexpr bool PRE = NR <= 4;
  C bv[PRE ? NR : 1], Dv[PRE ? NR : 1];
  auto load_bd = [&](int it, C& bb, C& dd) {
    const int k = min((int)threadIdx.x + 256 * it, RT - 1);
    const int a = k % RX, q = k / RX;
    int i0 = r0 + a, i1 = r1 + q % RY, i2 = r2 + q / RY;
    clamp_node(g, i0, i1, i2);
    const int f = flat(g, i0, i1, i2);
    bb = conv<C>::from(b[f]);
    dd = XIN ? op.diag(f, i0, i1, i2) : mk((R)0, (R)0);
  };
  if (PRE)
#pragma unroll
    for (int it = 0; it < (PRE ? NR : 1); ++it) load_bd(it, bv[it], Dv[it]);
  if (XIN) {
    stage_xin<DIM, XIN, SX, SY, SZ>(op, x, b, w_in, (const C*)nullptr, 1, 1, 0, 0, 0, r0 - 1, r1 - 1,
                                    DIM == 3 ? r2 - 1 : 0, xs);
    __syncthreads();
  }
  C rv[ALIAS ? NR : 1];
#pragma unroll(PRE || ALIAS ? NR : 4)
  for (int it = 0; it < NR; ++it) {
    const int k = (int)threadIdx.x + 256 * it;
    if (k >= RT) continue;
    C bb, dd;
    if (PRE) {
      bb = bv[PRE ? it : 0];
      dd = Dv[PRE ? it : 0];
    } else {
      load_bd(it, bb, dd);
    }
    const int a = k % RX, q = k / RX;
    const int i0 = r0 + a, i1 = r1 + q % RY, i2 = r2 + q / RY;
    C v = mk((R)0, (R)0);
    if (inside(g, i0, i1, i2)) {
      const int f = flat(g, i0, i1, i2);
      v = bb;
      if (XIN) {
        const int kk = (a + 1) + SX * ((q % RY + 1) + SY * (DIM == 3 ? q / RY + 1 : 0));
        v -= op.ax(xs, kk, SX, SX * SY, f, dd);
      }
    }
    if (ALIAS)
      rv[ALIAS ? it : 0] = v;
    else
      rs[k] = v;
  }
  if (ALIAS) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < (ALIAS ? NR : 0); ++it)
      if ((int)threadIdx.x + 256 * it < RT) rs[(int)threadIdx.x + 256 * it] = rv[it];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < CX * CY * CZ; k += 256) {
    const int a = k % CX, q = k / CX, bb = q % CY, cc = q / CY;
    const int I0 = O0 + a, I1 = O1 + bb, I2 = O2 + cc;
    if (!inside(g2, I0, I1, I2)) continue;
    C acc = mk((R)0, (R)0);
#pragma unroll
    for (int d2 = (DIM == 3 ? -1 : 0); d2 <= (DIM == 3 ? 1 : 0); ++d2) {
      const R w2 = DIM == 3 ? (d2 == 0 ? (R)0.5 : (R)0.25) : (R)1;
#pragma unroll
      for (int d1 = -1; d1 <= 1; ++d1) {
        const R w1 = d1 == 0 ? (R)0.5 : (R)0.25;
#pragma unroll
        for (int d0 = -1; d0 <= 1; ++d0) {
          const R w0 = d0 == 0 ? (R)0.5 : (R)0.25;
          const int kk = (2 * a + 1 + d0) + RX * ((2 * bb + 1 + d1) + RY * (DIM == 3 ? 2 * cc + 1 + d2 : 0));
          acc += (w0 * w1 * w2) * rs[kk];
        }
      }
    }
    b2[flat(g2, I0, I1, I2)] = acc;
  }
}

// ---- z-marching tiles (3D) --------------------------------------------------
// A block owns an xy tile and walks consecutive planes.  The staged iterate x_in lives in
// a ring of 4 planes (tile plus a one-node halo) in LDS; the inputs of the plane after
// next are requested into registers while the current plane is computed; the thread that
// stages a node keeps the b and D it loaded, and computes that node's output (sweep) or
// residual (restriction) from them.  Against the box tiles this stages about 1.2-1.4
// nodes per output instead of 2, loads b and D once instead of twice, and forms each
// slot's indices once per block.  The sums are those of the box kernels, in their order.
struct ZSlots {
  int k, fxy, j0, j1;    // staged position, flat xy offset and clamped coordinates
  bool in, own;          // xy inside the grid (and a real position); an output / residual node
};

template <class Op, typename CB, typename CO, int XIN, int BV>
__global__ void __launch_bounds__(256) k_sweep_z(Op op, const typename Op::C* __restrict__ x,
                                                 const CB* __restrict__ b, typename Op::Real w_in, Geom gc,
                                                 const typename Op::C* __restrict__ e, typename Op::Real w,
                                                 CO* __restrict__ out, TileGrid tg) {
  typedef typename Op::C C;
  typedef typename Op::Real R;
  typedef typename Op::Aux A;
  constexpr int TX = ZSBox<BV>::x, TY = ZSBox<BV>::y, ZC = ZSBox<BV>::z;
  constexpr int SX = TX + 2, SY = TY + 2, PL = SX * SY, NS = (PL + 255) / 256;
  constexpr int EX = TX / 2 + 3, EY = TY / 2 + 3, EZ = ZC / 2 + 3;
  __shared__ C ring[4 * PL];
  __shared__ C es[(XIN & XIN_E) ? EX * EY * EZ : 1];
  const Geom& g = op.geom();
  const long long ry = blockIdx.y;
  if (XIN & XIN_X) x += ry * g.tot;
  b += ry * g.tot;
  if (XIN & XIN_E) e += ry * gc.tot;
  out += ry * g.tot;
  int o0, o1, o2;
  if (!tile_origin(tg, TX, TY, ZC, o0, o1, o2)) return;
  const int s0 = o0 - 1, s1 = o1 - 1;
  const int c0 = s0 >> 1, c1 = s1 >> 1, c2 = (o2 - 1) >> 1;
  if (XIN & XIN_E) {
    constexpr int tot = EX * EY * EZ, NIT = (tot + 255) / 256;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int k = min((int)threadIdx.x + 256 * it, tot - 1);
      const int a = k % EX, q = k / EX;
      const int j0 = c0 + a, j1 = c1 + q % EY, j2 = c2 + q / EY;
      int l0 = j0, l1 = j1, l2 = j2;
      clamp_node(gc, l0, l1, l2);
      C v = e[flat(gc, l0, l1, l2)];
      if (!inside(gc, j0, j1, j2)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * it < tot) es[k] = v;
    }
    __syncthreads();
  }
  ZSlots sl[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int k = min((int)threadIdx.x + 256 * u, PL - 1);
    const int a = k % SX, q = k / SX;
    const int i0 = s0 + a, i1 = s1 + q;
    sl[u].k = k;
    sl[u].j0 = min(max(i0, 0), g.n[0]);
    sl[u].j1 = min(max(i1, 0), g.n[1]);
    sl[u].fxy = sl[u].j0 + g.N[0] * sl[u].j1;
    sl[u].in = (int)threadIdx.x + 256 * u < PL && i0 >= 0 && i0 <= g.n[0] && i1 >= 0 && i1 <= g.n[1];
    sl[u].own = sl[u].in && a >= 1 && a <= TX && q >= 1 && q <= TY;
  }
  const int NP = g.N[0] * g.N[1];
  // two register sets of plane inputs: plane q in set q & 1, requested two planes ahead
  C rx[2][NS];
  CB rb[2][NS];
  A ra[2][NS];
  auto load = [&](auto S, int z) {
    constexpr int s = decltype(S)::value;
    const int base = NP * min(max(z, 0), g.n[2]);
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int f = base + sl[u].fxy;
      if (XIN & XIN_X) rx[s][u] = x[f];
      rb[s][u] = b[f];
      ra[s][u] = op.aux(f);
    }
  };
  // x_in of plane z (inputs in set S) into its ring slot; bo, Do receive its b and D
  auto stage = [&](auto S, int z, C* bo, C* Do) {
    constexpr int s = decltype(S)::value;
    const int jz = min(max(z, 0), g.n[2]);
    const bool inz = z >= 0 && z <= g.n[2];
    C* dst = ring + (z & 3) * PL;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const C D = op.diag_aux(ra[s][u], sl[u].j0, sl[u].j1, jz);
      const C bb = conv<C>::from(rb[s][u]);
      C v = mk((R)0, (R)0);
      if (XIN & XIN_X) v += rx[s][u];
      if (XIN & XIN_Z) v += w_in * jdiv(bb, D);
      if (XIN & XIN_E) v += prolong_lds<3>(es, EX, EY, c0, c1, c2, sl[u].j0, sl[u].j1, jz);
      if (!(sl[u].in && inz)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * u < PL) dst[sl[u].k] = v;
      bo[u] = bb;
      Do[u] = D;
    }
  };
  const std::integral_constant<int, 0> S0;
  const std::integral_constant<int, 1> S1;
  const int zend = min(o2 + ZC, g.n[2] + 1);        // output planes o2 .. zend - 1 (o2 even)
  C bA[NS], DA[NS], bB[NS], DB[NS];
  load(S1, o2 - 1);
  stage(S1, o2 - 1, bA, DA);
  load(S0, o2);
  load(S1, o2 + 1);
  stage(S0, o2, bA, DA);
  load(S0, o2 + 2);
  // plane p: stage p + 1 (set S, = (p + 1) & 1), refill S with p + 3, output p
  auto plane = [&](auto S, int p) {
    stage(S, p + 1, bB, DB);
    if (p + 3 <= zend) load(S, p + 3);
    __syncthreads();
    const C* xm = ring + ((p - 1) & 3) * PL;
    const C* x0 = ring + (p & 3) * PL;
    const C* xp = ring + ((p + 1) & 3) * PL;
    const int base = NP * p;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      if (sl[u].own) {
        const int f = base + sl[u].fxy;
        const C r = bA[u] - op.ax3(xm, x0, xp, sl[u].k, SX, f, DA[u]);
        out[f] = conv<CO>::from(x0[sl[u].k] + w * jdiv(r, DA[u]));
      }
      bA[u] = bB[u];
      DA[u] = DB[u];
    }
  };
  for (int p = o2; p < zend; p += 2) {
    plane(S1, p);
    if (p + 1 < zend) plane(S0, p + 1);
  }
}

// b_c(I) = sum_f R(I, f) (b - A x_in)(f) over a coarse xy tile and CZ coarse planes: the
// fine residual planes 2 Z - 1, 2 Z, 2 Z + 1 of coarse plane Z arrive in that order, and
// each coarse node's sum takes their terms in the box kernel's order (one accumulator for
// plane Z, one started for Z + 1 by the odd plane they share)
template <class Op, typename CB, int XIN, int BV>
__global__ void __launch_bounds__(256) k_restrict_z(Op op, const typename Op::C* __restrict__ x,
                                                    const CB* __restrict__ b, typename Op::Real w_in, Geom g2,
                                                    typename Op::C* __restrict__ b2, TileGrid tg) {
  typedef typename Op::C C;
  typedef typename Op::Real R;
  typedef typename Op::Aux A;
  constexpr int CX = ZRBox<BV>::x, CY = ZRBox<BV>::y, CZ = ZRBox<BV>::z;
  constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1;
  constexpr int SX = RX + 2, SY = RY + 2, PL = SX * SY, NS = (PL + 255) / 256;
  static_assert(CX * CY <= 256, "one coarse node per thread");
  __shared__ C ring[4 * PL];
  __shared__ C rbuf[2 * PL];
  const Geom& g = op.geom();
  const long long ry = blockIdx.y;
  if (XIN & XIN_X) x += ry * g.tot;
  b += ry * g.tot;
  b2 += ry * g2.tot;
  int O0, O1, O2;
  if (!tile_origin(tg, CX, CY, CZ, O0, O1, O2)) return;
  const int s0 = 2 * O0 - 2, s1 = 2 * O1 - 2;       // staged region: residual region - 1
  ZSlots sl[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int k = min((int)threadIdx.x + 256 * u, PL - 1);
    const int a = k % SX, q = k / SX;
    const int i0 = s0 + a, i1 = s1 + q;
    sl[u].k = k;
    sl[u].j0 = min(max(i0, 0), g.n[0]);
    sl[u].j1 = min(max(i1, 0), g.n[1]);
    sl[u].fxy = sl[u].j0 + g.N[0] * sl[u].j1;
    sl[u].in = (int)threadIdx.x + 256 * u < PL && i0 >= 0 && i0 <= g.n[0] && i1 >= 0 && i1 <= g.n[1];
    sl[u].own = (int)threadIdx.x + 256 * u < PL && a >= 1 && a <= RX && q >= 1 && q <= RY;
  }
  const int NP = g.N[0] * g.N[1];
  // two register sets of plane inputs: plane q in set q & 1, requested two planes ahead
  C rx[2][NS];
  CB rb[2][NS];
  A ra[2][NS];
  auto load = [&](auto S, int z) {
    constexpr int s = decltype(S)::value;
    const int base = NP * min(max(z, 0), g.n[2]);
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int f = base + sl[u].fxy;
      if (XIN & XIN_X) rx[s][u] = x[f];
      rb[s][u] = b[f];
      ra[s][u] = op.aux(f);
    }
  };
  auto stage = [&](auto S, int z, C* bo, C* Do) {
    constexpr int s = decltype(S)::value;
    const int jz = min(max(z, 0), g.n[2]);
    const bool inz = z >= 0 && z <= g.n[2];
    C* dst = ring + (z & 3) * PL;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const C D = op.diag_aux(ra[s][u], sl[u].j0, sl[u].j1, jz);
      const C bb = conv<C>::from(rb[s][u]);
      C v = mk((R)0, (R)0);
      if (XIN & XIN_X) v += rx[s][u];
      if (XIN & XIN_Z) v += w_in * jdiv(bb, D);
      if (!(sl[u].in && inz)) v = mk((R)0, (R)0);
      if ((int)threadIdx.x + 256 * u < PL) dst[sl[u].k] = v;
      bo[u] = bb;
      Do[u] = D;
    }
  };
  const std::integral_constant<int, 0> S0;
  const std::integral_constant<int, 1> S1;
  // this thread's coarse node
  const int t = threadIdx.x;
  const bool cown = t < CX * CY;
  const int ca = t % CX, cb = t / CX;
  const bool cin = cown && O0 + ca <= g2.n[0] && O1 + cb <= g2.n[1];
  const int zc_end = min(O2 + CZ, g2.n[2] + 1);      // coarse planes O2 .. zc_end - 1
  const int p0 = 2 * O2 - 1, p1 = 2 * zc_end - 1;    // fine residual planes p0 .. p1 (p0 odd)
  C accA = mk((R)0, (R)0), accB = mk((R)0, (R)0);
  C bA[NS], DA[NS], bB[NS], DB[NS];
  load(S0, p0 - 1);
  stage(S0, p0 - 1, bA, DA);
  load(S1, p0);
  load(S0, p0 + 1);
  stage(S1, p0, bA, DA);
  load(S1, p0 + 2);
  // residual plane p: stage p + 1 (set S, = (p + 1) & 1), refill S with p + 3
  auto plane = [&](auto S, int p) {
    stage(S, p + 1, bB, DB);
    if (p + 3 <= p1 + 1) load(S, p + 3);
    __syncthreads();
    const C* xm = ring + ((p - 1) & 3) * PL;
    const C* x0 = ring + (p & 3) * PL;
    const C* xp = ring + ((p + 1) & 3) * PL;
    C* rs = rbuf + (p & 1) * PL;
    const bool inz = p >= 0 && p <= g.n[2];
    const int base = NP * p;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      if (sl[u].own) {
        C v = mk((R)0, (R)0);
        if (sl[u].in && inz) {
          v = bA[u];
          if (XIN) v -= op.ax3(xm, x0, xp, sl[u].k, SX, base + sl[u].fxy, DA[u]);
        }
        rs[sl[u].k] = v;
      }
      bA[u] = bB[u];
      DA[u] = DB[u];
    }
    __syncthreads();
    if (cown) {
      // the 3 x 3 in-plane terms of this residual plane, weights w0 w1 w2 as in k_restrict
      auto terms = [&](C acc, R w2) {
#pragma unroll
        for (int d1 = -1; d1 <= 1; ++d1) {
          const R w1 = d1 == 0 ? (R)0.5 : (R)0.25;
#pragma unroll
          for (int d0 = -1; d0 <= 1; ++d0) {
            const R w0 = d0 == 0 ? (R)0.5 : (R)0.25;
            acc += (w0 * w1 * w2) * rs[(2 * ca + 2 + d0) + SX * (2 * cb + 2 + d1)];
          }
        }
        return acc;
      };
      if ((p & 1) == 0) {
        accA = terms(accA, (R)0.5);                  // d2 = 0 of plane p / 2
      } else {
        const int Z = (p - 1) >> 1;                  // d2 = +1 of Z, then d2 = -1 of Z + 1
        if (Z >= O2) {
          accA = terms(accA, (R)0.25);
          if (cin) b2[flat(g2, O0 + ca, O1 + cb, Z)] = accA;
        }
        if (Z + 1 < zc_end) accB = terms(mk((R)0, (R)0), (R)0.25);
        accA = accB;
      }
    }
  };
  for (int p = p0; p <= p1; p += 2) {
    plane(S0, p);
    if (p + 1 <= p1) plane(S1, p + 1);
  }
}

// ---- level-2 chain (2D) ------------------------------------------------------
// Between two level-2 visits with one pre- and one post-sweep, three kernels run back to
// back on level 2 with no coarse work between them: the post-sweep of the visit just ended
// (x_in = x or the virtual first sweep, plus the coarse correction e), the pre-sweep of the
// next visit, and that visit's residual and restriction.  One coarse box of this kernel
// does all three on its fine footprint: the virtual iterate x0 on the footprint plus a
// halo of 3, xa = one Jacobi sweep of x0 on halo 2, xb = one sweep of xa on halo 1 (written
// for the box's own fine nodes [2 O, 2 O + 2 C)), r = b - A xb on the footprint and
// b3 = R r.  The sums are those of k_sweep and k_restrict, in their order.
template <class Op, int XIN>
__global__ void __launch_bounds__(256) k_l2_chain(Op op, const typename Op::C* __restrict__ x,
                                                  const typename Op::C* __restrict__ b, typename Op::Real w_in,
                                                  Geom gc, const typename Op::C* __restrict__ e, typename Op::Real w,
                                                  typename Op::C* __restrict__ xb_out, typename Op::C* __restrict__ b3,
                                                  TileGrid tg) {
  typedef typename Op::C C;
  typedef typename Op::Real R;
  constexpr int CX = RBox<2, 0>::x, CY = RBox<2, 0>::y;
  constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1;           // residual footprint
  constexpr int AX = RX + 6, AY = RY + 6;                   // x0: halo 3
  constexpr int BX = RX + 4, BY = RY + 4;                   // xa: halo 2
  constexpr int DX = RX + 2, DY = RY + 2;                   // xb: halo 1
  constexpr int EX = AX / 2 + 2, EY = AY / 2 + 2;           // e on x0's coarse footprint
  __shared__ C es[EX * EY];
  __shared__ C x0[AX * AY];
  __shared__ C xa[BX * BY];
  __shared__ C xb[DX * DY];
  __shared__ C rs[RX * RY];
  const Geom& g = op.geom();
  const long long ry = blockIdx.y;
  if (XIN & XIN_X) x += ry * g.tot;
  b += ry * g.tot;
  e += ry * gc.tot;
  xb_out += ry * g.tot;
  b3 += ry * gc.tot;
  int O0, O1, O2;
  if (!tile_origin(tg, CX, CY, 1, O0, O1, O2)) return;
  const int f0 = 2 * O0 - 1, f1 = 2 * O1 - 1;               // the footprint's origin
  const int c0 = (f0 - 3) >> 1, c1 = (f1 - 3) >> 1;         // floor: may be negative
  for (int k = threadIdx.x; k < EX * EY; k += 256) {
    const int j0 = c0 + k % EX, j1 = c1 + k / EX;
    int l0 = j0, l1 = j1, l2 = 0;
    clamp_node(gc, l0, l1, l2);
    C v = e[flat(gc, l0, l1, 0)];
    if (!inside(gc, j0, j1, 0)) v = mk((R)0, (R)0);
    es[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < AX * AY; k += 256) {
    const int i0 = f0 - 3 + k % AX, i1 = f1 - 3 + k / AX;
    int j0 = i0, j1 = i1, j2 = 0;
    clamp_node(g, j0, j1, j2);
    const int f = flat(g, j0, j1, 0);
    C v = prolong_lds<2>(es, EX, EY, c0, c1, 0, j0, j1, 0);
    if (XIN & XIN_X) v += x[f];
    if (XIN & XIN_Z) v += w_in * jdiv(b[f], op.diag(f, j0, j1, 0));
    if (!inside(g, i0, i1, 0)) v = mk((R)0, (R)0);
    x0[k] = v;
  }
  __syncthreads();
  // one Jacobi sweep from src (stride sx, the node's centre at (a + 1, q + 1)) into dst
  auto sweep = [&](const C* src, int sx, C* dst, int nx, int ny, int o0, int o1, bool write_out) {
    for (int k = threadIdx.x; k < nx * ny; k += 256) {
      const int a = k % nx, q = k / nx;
      const int i0 = o0 + a, i1 = o1 + q;
      C v = mk((R)0, (R)0);
      if (inside(g, i0, i1, 0)) {
        const int f = flat(g, i0, i1, 0);
        const C D = op.diag(f, i0, i1, 0);
        const int kk = (a + 1) + sx * (q + 1);
        const C r = b[f] - op.ax(src, kk, sx, 0, f, D);
        v = src[kk] + w * jdiv(r, D);
        if (write_out && i0 >= 2 * O0 && i0 < 2 * (O0 + CX) && i1 >= 2 * O1 && i1 < 2 * (O1 + CY)) xb_out[f] = v;
      }
      dst[k] = v;
    }
  };
  sweep(x0, AX, xa, BX, BY, f0 - 2, f1 - 2, false);
  __syncthreads();
  sweep(xa, BX, xb, DX, DY, f0 - 1, f1 - 1, true);
  __syncthreads();
  for (int k = threadIdx.x; k < RX * RY; k += 256) {
    const int a = k % RX, q = k / RX;
    const int i0 = f0 + a, i1 = f1 + q;
    C v = mk((R)0, (R)0);
    if (inside(g, i0, i1, 0)) {
      const int f = flat(g, i0, i1, 0);
      const C D = op.diag(f, i0, i1, 0);
      v = b[f];
      v -= op.ax(xb, (a + 1) + DX * (q + 1), DX, 0, f, D);
    }
    rs[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < CX * CY; k += 256) {
    const int a = k % CX, q = k / CX;
    const int I0 = O0 + a, I1 = O1 + q;
    if (!inside(gc, I0, I1, 0)) continue;
    C acc = mk((R)0, (R)0);
#pragma unroll
    for (int d1 = -1; d1 <= 1; ++d1) {
      const R w1 = d1 == 0 ? (R)0.5 : (R)0.25;
#pragma unroll
      for (int d0 = -1; d0 <= 1; ++d0) {
        const R w0 = d0 == 0 ? (R)0.5 : (R)0.25;
        acc += (w0 * w1 * (R)1) * rs[(2 * a + 1 + d0) + RX * (2 * q + 1 + d1)];
      }
    }
    b3[flat(gc, I0, I1, 0)] = acc;
  }
}

// ---- cycle tail (2D) -------------------------------------------------------------
// The last level-2 post-sweep (from x2 + P e3) feeds only the level-1 post-sweep (from
// w D1^-1 b1 + P e2): one level-1 box of this kernel computes the level-2 sweep on the
// coarse footprint its staging reads (plus a halo of 1 for the sweep's neighbours) and then
// the level-1 sweep, so the level-2 iterate is never written.  The sums are those of
// k_sweep on each level, in its order.
template <typename R, typename CO>
__global__ void __launch_bounds__(256) k_cycle_tail(Op1<2, R> o1, Op2<2, R> o2, const cd* __restrict__ b1, R w1,
                                                    const typename cplx<R>::type* __restrict__ x2,
                                                    const typename cplx<R>::type* __restrict__ b2, R w2, Geom g3,
                                                    const typename cplx<R>::type* __restrict__ e3,
                                                    CO* __restrict__ out, TileGrid tg) {
  typedef typename cplx<R>::type C;
  constexpr int TX = SBox<2, 0>::x, TY = SBox<2, 0>::y;
  constexpr int SX = TX + 2, SY = TY + 2;                   // level-1 staging
  constexpr int EX = TX / 2 + 3, EY = TY / 2 + 3;           // e2 on its coarse footprint
  constexpr int YX = EX + 2, YY = EY + 2;                   // x2 + P e3 on that plus a halo of 1
  constexpr int FX = YX / 2 + 2, FY = YY / 2 + 2;           // e3 on the level-3 footprint
  __shared__ C e3s[FX * FY];
  __shared__ C y2[YX * YY];
  __shared__ C e2s[EX * EY];
  __shared__ C xs[SX * SY];
  const Geom& g1 = o1.geom();
  const Geom& g2 = o2.geom();
  const long long ry = blockIdx.y;
  b1 += ry * g1.tot;
  out += ry * g1.tot;
  x2 += ry * g2.tot;
  b2 += ry * g2.tot;
  e3 += ry * g3.tot;
  int o0, o1_, o2_;
  if (!tile_origin(tg, TX, TY, 1, o0, o1_, o2_)) return;
  const int s0 = o0 - 1, s1 = o1_ - 1;
  const int c0 = s0 >> 1, c1 = s1 >> 1;                     // floor: may be negative
  const int q0 = c0 - 1, q1 = c1 - 1;
  const int d0 = q0 >> 1, d1 = q1 >> 1;
  for (int k = threadIdx.x; k < FX * FY; k += 256) {
    const int j0 = d0 + k % FX, j1 = d1 + k / FX;
    int l0 = j0, l1 = j1, l2 = 0;
    clamp_node(g3, l0, l1, l2);
    C v = e3[flat(g3, l0, l1, 0)];
    if (!inside(g3, j0, j1, 0)) v = mk((R)0, (R)0);
    e3s[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < YX * YY; k += 256) {
    const int i0 = q0 + k % YX, i1 = q1 + k / YX;
    int j0 = i0, j1 = i1, j2 = 0;
    clamp_node(g2, j0, j1, j2);
    C v = prolong_lds<2>(e3s, FX, FY, d0, d1, 0, j0, j1, 0);
    v += x2[flat(g2, j0, j1, 0)];
    if (!inside(g2, i0, i1, 0)) v = mk((R)0, (R)0);
    y2[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < EX * EY; k += 256) {
    const int a = k % EX, q = k / EX;
    const int i0 = c0 + a, i1 = c1 + q;
    C v = mk((R)0, (R)0);
    if (inside(g2, i0, i1, 0)) {
      const int f = flat(g2, i0, i1, 0);
      const C D = o2.diag(f, i0, i1, 0);
      const int kk = (a + 1) + YX * (q + 1);
      const C r = b2[f] - o2.ax(y2, kk, YX, 0, f, D);
      v = y2[kk] + w2 * jdiv(r, D);
    }
    e2s[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < SX * SY; k += 256) {
    const int i0 = s0 + k % SX, i1 = s1 + k / SX;
    int j0 = i0, j1 = i1, j2 = 0;
    clamp_node(g1, j0, j1, j2);
    const int f = flat(g1, j0, j1, 0);
    C v = prolong_lds<2>(e2s, EX, EY, c0, c1, 0, j0, j1, 0);
    v += w1 * jdiv(conv<C>::from(b1[f]), o1.diag(f, j0, j1, 0));
    if (!inside(g1, i0, i1, 0)) v = mk((R)0, (R)0);
    xs[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < TX * TY; k += 256) {
    const int a = k % TX, q = k / TX;
    const int i0 = o0 + a, i1 = o1_ + q;
    if (!inside(g1, i0, i1, 0)) continue;
    const int f = flat(g1, i0, i1, 0);
    const C bo = conv<C>::from(b1[f]);
    const C D = o1.diag(f, i0, i1, 0);
    const int kk = (a + 1) + SX * (q + 1);
    const C r = bo - o1.ax(xs, kk, SX, 0, f, D);
    out[f] = conv<CO>::from(xs[kk] + w1 * jdiv(r, D));
  }
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

// ------------------------------- launchers ---------------------------------
static inline unsigned grid_for(long long n) { return (unsigned)((n + 255) / 256); }
static inline unsigned grid_xcd(long long n) {
  long long nb = (n + 255) / 256;
  long long per = (nb + 7) / 8;
  return (unsigned)(per * 8);
}
static inline TileGrid tiles(const Geom& g, int bx, int by, int bz) {
  TileGrid t;
  t.nt[0] = (g.N[0] + bx - 1) / bx;
  t.nt[1] = (g.N[1] + by - 1) / by;
  t.nt[2] = (g.N[2] + bz - 1) / bz;
  t.ntiles = t.nt[0] * t.nt[1] * t.nt[2];
  return t;
}
static inline unsigned grid_tiles(const TileGrid& t) { return (unsigned)((t.ntiles + 7) / 8 * 8); }

template <int DIM, class Op, typename CB, typename CO, int BV>
void sweep_box(const Op& op, int xin, const typename Op::C* x, const CB* b, typename Op::Real w_in,
               const Geom& gc, const typename Op::C* e, typename Op::Real w, CO* out, int nrhs, hipStream_t s) {
  TileGrid tg = tiles(op.geom(), SBox<DIM, BV>::x, SBox<DIM, BV>::y, SBox<DIM, BV>::z);
  dim3 grid(grid_tiles(tg), nrhs), blk(256);
#define SW(F) \
  hipLaunchKernelGGL((k_sweep<DIM, Op, CB, CO, F, BV>), grid, blk, 0, s, op, x, b, w_in, gc, e, w, out, tg)
  switch (xin) {
    case 0: SW(0); break;
    case XIN_X: SW(XIN_X); break;
    case XIN_Z: SW(XIN_Z); break;
    case XIN_E: SW(XIN_E); break;
    case XIN_X | XIN_E: SW(XIN_X | XIN_E); break;
    case XIN_Z | XIN_E: SW(XIN_Z | XIN_E); break;
    default: break;
  }
#undef SW
}

template <class Op, typename CB, typename CO, int BV>
void sweep_z(const Op& op, int xin, const typename Op::C* x, const CB* b, typename Op::Real w_in, const Geom& gc,
             const typename Op::C* e, typename Op::Real w, CO* out, int nrhs, hipStream_t s) {
  TileGrid tg = tiles(op.geom(), ZSBox<BV>::x, ZSBox<BV>::y, ZSBox<BV>::z);
  dim3 grid(grid_tiles(tg), nrhs), blk(256);
#define SW(F) hipLaunchKernelGGL((k_sweep_z<Op, CB, CO, F, BV>), grid, blk, 0, s, op, x, b, w_in, gc, e, w, out, tg)
  switch (xin) {
    case XIN_X: SW(XIN_X); break;
    case XIN_Z: SW(XIN_Z); break;
    case XIN_E: SW(XIN_E); break;
    case XIN_X | XIN_E: SW(XIN_X | XIN_E); break;
    case XIN_Z | XIN_E: SW(XIN_Z | XIN_E); break;
    default: break;
  }
#undef SW
}

template <int DIM, class Op, typename CB, typename CO>
void sweep_dim(const Op& op, int xin, const typename Op::C* x, const CB* b, typename Op::Real w_in,
               const Geom& gc, const typename Op::C* e, typename Op::Real w, CO* out, int nrhs, hipStream_t s) {
  // the FP64 cycle's 3D boxes stay at variant 0 (the larger ones exceed the block's LDS);
  // the z-marching variants are 3D (variant 0 in 2D), and a sweep from nothing (xin 0,
  // which materialises zero) keeps the box kernel
  const int v = (DIM == 3 && sizeof(typename Op::C) == 16) ? 0 : op.A.box_sweep;
  if constexpr (DIM == 3 && sizeof(typename Op::C) == 16) {
    sweep_box<DIM, Op, CB, CO, 0>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s);
  } else if constexpr (DIM == 3) {
    switch (xin == 0 ? 0 : v) {
      case 1: sweep_box<DIM, Op, CB, CO, 1>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      case 2: sweep_box<DIM, Op, CB, CO, 2>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      case 3: sweep_box<DIM, Op, CB, CO, 3>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      case 4: sweep_z<Op, CB, CO, 4>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      case 5: sweep_z<Op, CB, CO, 5>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      default: sweep_box<DIM, Op, CB, CO, 0>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
    }
  } else {
    switch (v) {
      case 1: sweep_box<DIM, Op, CB, CO, 1>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      case 2: sweep_box<DIM, Op, CB, CO, 2>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      case 3: sweep_box<DIM, Op, CB, CO, 3>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
      default: sweep_box<DIM, Op, CB, CO, 0>(op, xin, x, b, w_in, gc, e, w, out, nrhs, s); break;
    }
  }
}

template <int DIM, class Op, typename CB, int BV>
void restrict_box(const Op& op, int xin, const typename Op::C* x, const CB* b, typename Op::Real w_in,
                  const Geom& g2, typename Op::C* b2, int nrhs, hipStream_t s) {
  TileGrid tg = tiles(g2, RBox<DIM, BV>::x, RBox<DIM, BV>::y, RBox<DIM, BV>::z);
  dim3 grid(grid_tiles(tg), nrhs), blk(256);
#define RS(F) hipLaunchKernelGGL((k_restrict<DIM, Op, CB, F, BV>), grid, blk, 0, s, op, x, b, w_in, g2, b2, tg)
  switch (xin) {
    case 0: RS(0); break;
    case XIN_X: RS(XIN_X); break;
    case XIN_Z: RS(XIN_Z); break;
    default: break;
  }
#undef RS
}

template <class Op, typename CB, int BV>
void restrict_z(const Op& op, int xin, const typename Op::C* x, const CB* b, typename Op::Real w_in,
                const Geom& g2, typename Op::C* b2, int nrhs, hipStream_t s) {
  TileGrid tg = tiles(g2, ZRBox<BV>::x, ZRBox<BV>::y, ZRBox<BV>::z);
  dim3 grid(grid_tiles(tg), nrhs), blk(256);
  if (xin == XIN_X)
    hipLaunchKernelGGL((k_restrict_z<Op, CB, XIN_X, BV>), grid, blk, 0, s, op, x, b, w_in, g2, b2, tg);
  else if (xin == XIN_Z)
    hipLaunchKernelGGL((k_restrict_z<Op, CB, XIN_Z, BV>), grid, blk, 0, s, op, x, b, w_in, g2, b2, tg);
}

template <int DIM, class Op, typename CB>
void restrict_dim(const Op& op, int xin, const typename Op::C* x, const CB* b, typename Op::Real w_in,
                  const Geom& g2, typename Op::C* b2, int nrhs, hipStream_t s) {
  if constexpr (DIM == 3 && sizeof(typename Op::C) == 16) {
    restrict_box<DIM, Op, CB, 0>(op, xin, x, b, w_in, g2, b2, nrhs, s);
  } else if constexpr (DIM == 3) {
    // the z-marching variants take an iterate (xin X or Z); restricting b alone keeps the
    // box kernel
    switch (xin == 0 ? 0 : op.A.box_restrict) {
      case 1: restrict_box<DIM, Op, CB, 1>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
      case 2: restrict_box<DIM, Op, CB, 2>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
      case 3: restrict_z<Op, CB, 3>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
      case 4: restrict_z<Op, CB, 4>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
      default: restrict_box<DIM, Op, CB, 0>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
    }
  } else {
    switch (op.A.box_restrict) {
      case 1: restrict_box<DIM, Op, CB, 1>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
      case 2: restrict_box<DIM, Op, CB, 2>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
      default: restrict_box<DIM, Op, CB, 0>(op, xin, x, b, w_in, g2, b2, nrhs, s); break;
    }
  }
}

template <typename R, typename CB, typename CO>
void l1_sweep(const L1<R>& A, int xin, const typename cplx<R>::type* x, const CB* b, R w_in, const Geom& gc,
              const typename cplx<R>::type* e, R w, CO* out, int nrhs, hipStream_t s) {
  if (A.op.g.dim == 2)
    sweep_dim<2>(Op1<2, R>{A}, xin, x, b, w_in, gc, e, w, out, nrhs, s);
  else
    sweep_dim<3>(Op1<3, R>{A}, xin, x, b, w_in, gc, e, w, out, nrhs, s);
}

template <typename R, typename CB>
void l1_restrict(const L1<R>& A, int xin, const typename cplx<R>::type* x, const CB* b, R w_in, const Geom& gc,
                 const typename cplx<R>::type* e, const Geom& g2, typename cplx<R>::type* b2, int nrhs,
                 hipStream_t s) {
  (void)gc;
  (void)e;
  if (A.op.g.dim == 2)
    restrict_dim<2>(Op1<2, R>{A}, xin, x, b, w_in, g2, b2, nrhs, s);
  else
    restrict_dim<3>(Op1<3, R>{A}, xin, x, b, w_in, g2, b2, nrhs, s);
}

template <typename R>
void l2_sweep(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b, R w_in,
              const Geom& gc, const typename cplx<R>::type* e, R w, typename cplx<R>::type* out, int nrhs,
              hipStream_t s) {
  typedef typename cplx<R>::type C;
  if (A.g.dim == 2)
    sweep_dim<2, Op2<2, R>, C, C>(Op2<2, R>{A}, xin, x, b, w_in, gc, e, w, out, nrhs, s);
  else
    sweep_dim<3, Op2<3, R>, C, C>(Op2<3, R>{A}, xin, x, b, w_in, gc, e, w, out, nrhs, s);
}

template <typename R>
void l2_restrict(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b,
                 R w_in, const Geom& gc, const typename cplx<R>::type* e, const Geom& g3,
                 typename cplx<R>::type* b3, int nrhs, hipStream_t s) {
  typedef typename cplx<R>::type C;
  (void)gc;
  (void)e;
  if (A.g.dim == 2)
    restrict_dim<2, Op2<2, R>, C>(Op2<2, R>{A}, xin, x, b, w_in, g3, b3, nrhs, s);
  else
    restrict_dim<3, Op2<3, R>, C>(Op2<3, R>{A}, xin, x, b, w_in, g3, b3, nrhs, s);
}

template <typename R, typename CO>
void cycle_tail(const L1<R>& A1, const cd* b1, R w1, const L2<R>& A2, const typename cplx<R>::type* x2,
                const typename cplx<R>::type* b2, R w2, const Geom& g3, const typename cplx<R>::type* e3, CO* out,
                int nrhs, hipStream_t s) {
  TileGrid tg = tiles(A1.op.g, SBox<2, 0>::x, SBox<2, 0>::y, 1);
  dim3 grid(grid_tiles(tg), nrhs), blk(256);
  hipLaunchKernelGGL((k_cycle_tail<R, CO>), grid, blk, 0, s, Op1<2, R>{A1}, Op2<2, R>{A2}, b1, w1, x2, b2, w2, g3, e3,
                     out, tg);
}

template <typename R>
void l2_chain(const L2<R>& A, int xin, const typename cplx<R>::type* x, const typename cplx<R>::type* b, R w_in,
              const Geom& gc, const typename cplx<R>::type* e, R w, typename cplx<R>::type* xb,
              typename cplx<R>::type* b3, int nrhs, hipStream_t s) {
  TileGrid tg = tiles(gc, RBox<2, 0>::x, RBox<2, 0>::y, 1);
  dim3 grid(grid_tiles(tg), nrhs), blk(256);
  if (xin == (XIN_Z | XIN_E))
    hipLaunchKernelGGL((k_l2_chain<Op2<2, R>, XIN_Z | XIN_E>), grid, blk, 0, s, Op2<2, R>{A}, x, b, w_in, gc, e, w,
                       xb, b3, tg);
  else
    throw std::runtime_error("l2_chain: the chain starts from the virtual first sweep (xin Z | E)");
}

void l1_apply64(const L1<double>& A, const void* x, int x_is_f32, cd* y, hipStream_t s) {
  dim3 grid(grid_xcd(A.op.g.tot)), blk(256);
  if (x_is_f32)
    hipLaunchKernelGGL((k_l1_apply64<cf>), grid, blk, 0, s, A, (const cf*)x, y);
  else
    hipLaunchKernelGGL((k_l1_apply64<cd>), grid, blk, 0, s, A, (const cd*)x, y);
}

__global__ void __launch_bounds__(256) k_l1_diag32(L1<float> A, cf* __restrict__ dg) {
  const Geom& g = A.op.g;
  for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < g.tot;
       f += (long long)gridDim.x * blockDim.x) {
    int i0, i1, i2;
    decode(g, f, i0, i1, i2);
    dg[f] = A.diag(f, i0, i1, i2);
  }
}

void l1_diag32(const L1<float>& A, cf* dg, hipStream_t s) {
  hipLaunchKernelGGL(k_l1_diag32, dim3(2048), dim3(256), 0, s, A, dg);
}

void l1_apply32(const L1<float>& A, const cf* x, cf* y, hipStream_t s) {
  dim3 grid(grid_xcd(A.op.g.tot)), blk(256);
  hipLaunchKernelGGL(k_l1_apply32, grid, blk, 0, s, A, x, y);
}

// explicit instantiations used by the cycle driver
template void l1_sweep<float, cd, cf>(const L1<float>&, int, const cf*, const cd*, float,
                                               const Geom&, const cf*, float, cf*, int, hipStream_t);
template void l1_sweep<float, cd, cd>(const L1<float>&, int, const cf*, const cd*, float,
                                                const Geom&, const cf*, float, cd*, int, hipStream_t);
template void l1_sweep<double, cd, cd>(const L1<double>&, int, const cd*, const cd*, double,
                                                 const Geom&, const cd*, double, cd*, int, hipStream_t);
template void l1_restrict<float, cd>(const L1<float>&, int, const cf*, const cd*, float,
                                          const Geom&, const cf*, const Geom&, cf*, int, hipStream_t);
template void l1_restrict<double, cd>(const L1<double>&, int, const cd*, const cd*, double,
                                           const Geom&, const cd*, const Geom&, cd*, int, hipStream_t);
template void l2_sweep<float>(const L2<float>&, int, const cf*, const cf*, float, const Geom&,
                              const cf*, float, cf*, int, hipStream_t);
template void l2_sweep<double>(const L2<double>&, int, const cd*, const cd*, double, const Geom&,
                               const cd*, double, cd*, int, hipStream_t);
template void cycle_tail<float, cf>(const L1<float>&, const cd*, float, const L2<float>&, const cf*, const cf*,
                                    float, const Geom&, const cf*, cf*, int, hipStream_t);
template void cycle_tail<float, cd>(const L1<float>&, const cd*, float, const L2<float>&, const cf*, const cf*,
                                    float, const Geom&, const cf*, cd*, int, hipStream_t);
template void cycle_tail<double, cd>(const L1<double>&, const cd*, double, const L2<double>&, const cd*, const cd*,
                                     double, const Geom&, const cd*, cd*, int, hipStream_t);
template void l2_chain<float>(const L2<float>&, int, const cf*, const cf*, float, const Geom&, const cf*, float,
                              cf*, cf*, int, hipStream_t);
template void l2_chain<double>(const L2<double>&, int, const cd*, const cd*, double, const Geom&, const cd*, double,
                               cd*, cd*, int, hipStream_t);
template void l2_restrict<float>(const L2<float>&, int, const cf*, const cf*, float, const Geom&,
                                 const cf*, const Geom&, cf*, int, hipStream_t);
template void l2_restrict<double>(const L2<double>&, int, const cd*, const cd*, double, const Geom&,
                                  const cd*, const Geom&, cd*, int, hipStream_t);

}  // namespace helm
