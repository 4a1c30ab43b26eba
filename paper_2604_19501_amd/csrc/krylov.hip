// FP64 kernels of the outer right-preconditioned FGMRES (restarted).
//
// Per iteration j (basis V_0..V_j, z_j = M^{-1} V_j from the cycle), two passes over
// the basis:
//   k_arnoldi_dots    w = H z_j (FP64) and, reading every V_i once, partial sums of
//                     h1_i = <V_i, w>, the Gram column G_ij = <V_i, V_j> and ||w||^2
//   k_fin_givens      the sums, in a fixed order, one block per value; the block that
//                     stores the last of them then runs classical Gram-Schmidt with one
//                     re-orthogonalisation, the second projection taken from the Gram
//                     matrix instead of a second pass:
//                       h2 = V^H (w - V h1) = h1 - G h1,   c = h1 + h2 = H(:, j),
//                       h_{j+1,j}^2 = ||w - V c||^2 = ||w||^2 - 2 Re(c^H h1) + c^H G c;
//                     then the Givens rotation of the Hessenberg column, the residual
//                     estimate |g_{j+1}| / ||b|| and the convergence flag
//   k_arnoldi_update  V_{j+1} = (H z_j - V c) / h_{j+1,j}, recomputing H z_j (16 B per
//                     node) instead of storing and reloading w (32 B per node); its first
//                     block also packs the state for the host
// Because G holds the inner products of the stored vectors, any loss of orthogonality
// of V is corrected in the next column rather than accumulated.  Reductions are
// two-stage (per-block partials, then a fixed-order sum), so the results are bitwise
// reproducible run to run.
#include <cstddef>

#include "krylov.h"
#include "wide.h"

namespace helm {

// v + (v of the lane that DPP control ctrl selects), the moved value 0 in the rows outside
// rmask; a double moves as its two 32-bit halves
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, RMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RMASK, 0xf, false);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// sum of v over the 64-lane wavefront in a fixed order, returned to every lane.  DPP lane
// moves (pair swap, quad swap, half-row mirror, row mirror, then the broadcasts of lanes 15
// and 31 into the rows above) leave the sum in lane 63; no LDS traffic.
__device__ __forceinline__ double wsum1(double v) {
  v = dpp_add<0xB1, 0xf>(v);        // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);        // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);       // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);       // row_mirror: every lane of a row holds the row's sum
  v = dpp_add<0x142, 0xa>(v);       // row_bcast15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);       // row_bcast31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ cd wsum(cd v) { return mk(wsum1(v.x), wsum1(v.y)); }

// sum v over the 256-thread block; thread 0 writes it to *out
__device__ __forceinline__ void block_sum(cd v, cd* lds, cd* out) {
  v = wsum(v);
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
}

// the per-right-hand-side pointers of right-hand side blockIdx.y (kept apart from the
// argument block, which must stay in kernel-argument memory)
struct RhsPtr {
  cd* V;
  KrylovState* st;
  cd* part;
};
__device__ __forceinline__ RhsPtr at_rhs(const KrylovArgs& a) {
  const long long r = blockIdx.y;
  return RhsPtr{a.V + r * a.op.g.tot, a.st + r, a.part + r * a.pstride};
}

__device__ __forceinline__ long long node_of(int q) {
  return ((long long)blockIdx.x * KNPT + q) * 256 + threadIdx.x;
}

// CMP: the compact fourth-order operator (no conjugate form), a separate instantiation of
// every kernel that applies H: inlined into the 5/7-point kernels as a run-time branch it
// raised their register count from 116 to 152 and added a stack frame
template <int CMP, typename CX>
__device__ __forceinline__ cd apply_h(const KrylovArgs& a, const CX* __restrict__ x, long long f) {
  const Geom& g = a.op.g;
  int i0, i1, i2;
  node_coords(g, f, i0, i1, i2);
  if constexpr (CMP) {
    cd dg;
    return g.dim == 3 ? wide_row<3, double, CX>(a.op, a.s, a.m64, x, f, i0, i1, i2, false, dg)
                      : wide_row<2, double, CX>(a.op, a.s, a.m64, x, f, i0, i1, i2, false, dg);
  }
  double sig = layer_sigma(a.op, i0, i1, i2);
  double mm = a.m64[f];
  cd c = a.s * mk(mm, -mm * sig);
  if (a.conj) c.y = -c.y;
  cd D = mk(2.0 * g.dim * a.op.inv_h2 - c.x, -c.y);
  // neighbours outside the grid are read at f and weighted 0, so that every load is
  // issued unconditionally (loads under a branch are waited for one by one)
  long long s1 = g.N[0], s2 = (long long)g.N[0] * g.N[1];
  const bool b0 = i0 > 0, b1 = i0 < g.n[0], b2 = i1 > 0, b3 = i1 < g.n[1];
  cd x0 = to_d(x[f]);
  cd xa = to_d(x[b0 ? f - 1 : f]), xb = to_d(x[b1 ? f + 1 : f]);
  cd xc = to_d(x[b2 ? f - s1 : f]), xd = to_d(x[b3 ? f + s1 : f]);
  cd nb = (b0 ? 1.0 : 0.0) * xa + (b1 ? 1.0 : 0.0) * xb + (b2 ? 1.0 : 0.0) * xc + (b3 ? 1.0 : 0.0) * xd;
  if (g.dim == 3) {
    const bool b4 = i2 > 0, b5 = i2 < g.n[2];
    cd xe = to_d(x[b4 ? f - s2 : f]), xf = to_d(x[b5 ? f + s2 : f]);
    nb += (b4 ? 1.0 : 0.0) * xe + (b5 ? 1.0 : 0.0) * xf;
  }
  return D * x0 - a.op.inv_h2 * nb;
}

// wave-level partial sums of nv values, then one fixed-order sum over the 4 waves per value
__device__ __forceinline__ void store_partials(cd (*red)[2 * KMAXM + 3], int nv, cd* part, int pcap) {
  __syncthreads();
  for (int t = threadIdx.x; t < nv; t += 256)
    part[(long long)t * pcap + blockIdx.x] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

// w = H z_j (FP64); partials of <V_i, w> (values 0..j), <V_i, V_j> (values j+1..2j+1) and
// ||w||^2 (value 2j+2, real part).  Nodes past the end are clamped to the last node and
// weighted 0; basis vector i + 1 is loaded while vector i is reduced, and V_j, loaded
// first for the Gram column, serves as the last vector (read from memory once).  The
// V_0..V_{j-1} loads are non-temporal: the basis (about 17 MB per vector at 1025^2) is
// larger than the caches, and streaming it through them would displace what the cycle
// reuses (measured: 1 % more solves per second at 1025^2 with these loads non-temporal).
template <typename CZ, int CMP>
__global__ void __launch_bounds__(256) k_arnoldi_dots(KrylovArgs a, const CZ* __restrict__ z, int j) {
  __shared__ cd red[4][2 * KMAXM + 3];
  const RhsPtr p = at_rhs(a);
  z += blockIdx.y * a.op.g.tot;
  if (p.st->done) return;          // an iteration queued after convergence: nothing to do
  const long long N = a.op.g.tot;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long f[KNPT];
  double on[KNPT];
  for (int q = 0; q < KNPT; ++q) {
    long long t = node_of(q);
    on[q] = t < N ? 1.0 : 0.0;
    f[q] = t < N ? t : N - 1;
  }
  cd w[KNPT], vj[KNPT], nx[KNPT];
  for (int q = 0; q < KNPT; ++q) {
    vj[q] = on[q] * p.V[(long long)j * a.ldv + f[q]];
    if (j > 0) nx[q] = ld_nt(p.V + f[q]);
  }
  double nw = 0.0;
  for (int q = 0; q < KNPT; ++q) {
    w[q] = on[q] * apply_h<CMP>(a, z, f[q]);
    nw += abs2(w[q]);
  }
  for (int i = 0; i <= j; ++i) {
    // V_i: the prefetched vector, or V_j itself (the weights of clamped nodes are 0 in w
    // and vj, so their partial terms vanish either way)
    cd vi[KNPT];
    for (int q = 0; q < KNPT; ++q) vi[q] = i < j ? nx[q] : vj[q];
    if (i + 1 < j)                                                // uniform over the block
      for (int q = 0; q < KNPT; ++q) nx[q] = ld_nt(p.V + (long long)(i + 1) * a.ldv + f[q]);
    cd s1 = mk(0.0, 0.0), s2 = mk(0.0, 0.0);
    for (int q = 0; q < KNPT; ++q) {
      s1 += cmulc(vi[q], w[q]);
      s2 += cmulc(vi[q], vj[q]);
    }
    s1 = wsum(s1);
    s2 = wsum(s2);
    if (lane == 0) {
      red[wv][i] = s1;
      red[wv][j + 1 + i] = s2;
    }
  }
  cd t = wsum(mk(nw, 0.0));
  if (lane == 0) red[wv][2 * j + 2] = t;
  store_partials(red, 2 * j + 3, p.part, a.pcap);
}

// r = b - H x (FP64) into V_0; partials of (||r||^2, ||b||^2) in slot 0
template <int CMP>
__global__ void __launch_bounds__(256) k_residual(KrylovArgs a, const cd* __restrict__ x,
                                                  const cd* __restrict__ b) {
  __shared__ cd lds[4];
  const RhsPtr p = at_rhs(a);
  x += blockIdx.y * a.op.g.tot;
  b += blockIdx.y * a.op.g.tot;
  const long long N = a.op.g.tot;
  cd v = mk(0.0, 0.0);
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f < N) {
      cd res = b[f] - apply_h<CMP>(a, x, f);
      p.V[f] = res;
      v += mk(abs2(res), abs2(b[f]));
    }
  }
  block_sum(v, lds, p.part + blockIdx.x);
}

// this thread's share of a block-wide sum of src[0 .. n): entries threadIdx.x + 256 m in
// increasing m; up to 8 of them are loaded before any is summed, so that they are in
// flight together (the order of the sums is that of the plain loop)
__device__ __forceinline__ cd sum_strided(const cd* __restrict__ src, int n) {
  cd v = mk(0.0, 0.0);
  for (int b = threadIdx.x; b < n; b += 256 * 8) {
    cd w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b + 256 * u < n) w[u] = src[b + 256 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b + 256 * u < n) v += w[u];
  }
  return v;
}

// one block per value: dst[i] = sum over blocks of part[i] (dst: the state member at off)
__global__ void __launch_bounds__(256) k_fin_sum(KrylovArgs a, size_t off) {
  __shared__ cd lds[4];
  const RhsPtr p = at_rhs(a);
  cd* dst = (cd*)((char*)p.st + off);
  const int i = blockIdx.x;
  cd v = mk(0.0, 0.0);
  v = sum_strided(p.part + (long long)i * a.pcap, a.nblk);
  block_sum(v, lds, dst + i);
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

// the scalar block (bnorm .. hist) of state r into slot r of the host-mapped dst
__device__ __forceinline__ void pack_state(const KrylovState* st, char* dst, int r) {
  constexpr int W = (int)((offsetof(KrylovState, hist) - offsetof(KrylovState, bnorm)) / 4);
  const int* src = (const int*)((const char*)st + offsetof(KrylovState, bnorm));
  for (int q = threadIdx.x; q < W; q += blockDim.x) ((int*)dst)[r * W + q] = src[q];
}

static_assert(KMAXM <= 64, "one lane per row of the Arnoldi column");

// LDS of a column's finish: the column's sums, the Gram matrix, the rotations
struct GivensLds {
  cd sh1[KMAXM + 1], sg[KMAXM + 1], sc[KMAXM + 1], col[KMAXM + 2], ssn[KMAXM];
  double scs[KMAXM], r1[64], r2[64];
  cd sG[(KMAXM + 1) * (KMAXM + 1) + 1];     // the last entry: a sink for stores past the end
};
// the scalars of the serial part, held by lane 0
struct GivensScal {
  cd gj;
  double bnorm;
  int its, maxit;
};

// first part of the finish of Arnoldi column j: what earlier launches wrote (G(i, k) for
// i, k < j, the rotations of columns < j, the scalars of the serial part) into LDS and lane
// 0's registers.  The first wavefront issues every load of a batch before it stores any, so
// that their latencies overlap; a barrier of the caller precedes their use.
__device__ __forceinline__ void givens_stage(GivensLds& L, const KrylovState* st, int j, GivensScal& sc) {
  const int t = threadIdx.x, ld = KMAXM + 1;
  if (t >= 64) return;
  if (t == 0) {
    sc.gj = st->g[j];
    sc.bnorm = st->bnorm;
    sc.its = st->its;
    sc.maxit = st->maxit;
  }
  // rotations: lane t < KMAXM loads entry t whether or not t < j (the rest are unused),
  // stored after the Gram loads so that all of them are in flight together
  const double cs_t = st->cs[t];
  const cd sn_t = st->sn[t];
  const int nG = j * j;
  for (int e0 = t; e0 < nG; e0 += 64 * 8) {
    // loads and stores unconditional (past the end: entry e0 into the sink), so that the
    // loads are not sunk into the stores' branches
    cd v[8];
    int at[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 64 * u < nG ? e0 + 64 * u : e0;
      at[u] = (e % j) + ld * (e / j);
      v[u] = st->G[at[u]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (e0 + 64 * u >= nG) at[u] = (KMAXM + 1) * (KMAXM + 1);
      L.sG[at[u]] = v[u];
    }
  }
  L.scs[t] = cs_t;
  L.ssn[t] = sn_t;
}

// second part: the sums of k_arnoldi_dots (st->h1), then the column and its Givens update
// in one block (256 threads in k_fin_givens, 64 in k_givens), of which the first wavefront
// works (the others only meet the barriers).  Lane i owns row i of the Gram products; the
// serial part (rotations of the column) runs on lane 0 out of LDS.
__device__ __forceinline__ void givens_finish(GivensLds& L, const KrylovArgs& a, KrylovState* st, int j, double tol,
                                              const GivensScal& sc) {
  const int t = threadIdx.x < 64 ? (int)threadIdx.x : 1 << 20, ld = KMAXM + 1;
  double nw2 = 0.0;
  if (t == 0) nw2 = st->h1[2 * j + 2].x;
  if (t <= j) {                                // j < KMAXM <= 64: one row per lane
    const cd h = st->h1[t], g = st->h1[j + 1 + t];   // g = G(t, j) = <V_t, V_j>
    L.sh1[t] = h;
    L.sg[t] = g;
    L.sG[j + ld * t] = conjc(g);
    L.sG[t + ld * j] = g;                      // the diagonal entry as summed
  }
  __syncthreads();
  auto gik = [&](int i, int k) -> cd { return L.sG[i + ld * k]; };
  // c = h1 + (h1 - G h1)
  if (t <= j) {
    cd gh = mk(0.0, 0.0);
    for (int k = 0; k <= j; ++k) gh += gik(t, k) * L.sh1[k];
    L.sc[t] = (L.sh1[t] + L.sh1[t]) - gh;
  }
  __syncthreads();
  // Re(c^H h1) and c^H G c, per lane then summed in lane order
  double p1 = 0.0, p2 = 0.0;
  if (t <= j) {
    cd gc = mk(0.0, 0.0);
    for (int k = 0; k <= j; ++k) gc += gik(t, k) * L.sc[k];
    p1 = L.sc[t].x * L.sh1[t].x + L.sc[t].y * L.sh1[t].y;
    p2 = L.sc[t].x * gc.x + L.sc[t].y * gc.y;
  }
  if (t < 64) {
    L.r1[t] = p1;
    L.r2[t] = p2;
  }
  if (t <= j) {                                // column / row j of G for later columns
    st->G[t + ld * j] = L.sg[t];
    st->G[j + ld * t] = conjc(L.sg[t]);
  }
  __syncthreads();
  if (t == 0) {
    double ch = 0.0, cgc = 0.0;
    for (int i = 0; i <= j; ++i) {
      ch += L.r1[i];
      cgc += L.r2[i];
    }
    const double n2 = nw2 - 2.0 * ch + cgc;     // ||w - V c||^2
    const double hn = n2 > 0.0 ? sqrt(n2) : 0.0;
    // the formula subtracts quantities of size ||w||^2: when ||w - V c|| << ||w|| (w almost
    // in the span of the basis) its rounding error swamps the value, so the column's
    // h_{j+1,j} and the next basis vector cannot be trusted.  The column is kept (its
    // rotation uses hn, which only enters through c^2 + hn^2 there) and the cycle ends:
    // the solution is updated and the restart recomputes the true residual in FP64.
    const bool cancel = n2 < a.guard * nw2;
    cd* col = L.col;
    st->hnext = hn;
    // previous rotations on column (c_0 .. c_j, hn): rotation i mixes entry i, already
    // rotated by rotation i - 1 and carried in registers, with the untouched c_{i+1}; the
    // rotated entry i is stored and not read again here
    cd hi = L.sc[0];
    for (int i = 0; i < j; ++i) {
      const cd hi1 = L.sc[i + 1];
      col[i] = L.scs[i] * hi + L.ssn[i] * hi1;
      hi = L.scs[i] * hi1 - conjc(L.ssn[i]) * hi;
    }
    col[j] = hi;
    col[j + 1] = mk(hn, 0.0);
    double c;
    cd s, r;
    givens(col[j], col[j + 1], c, s, r);
    st->cs[j] = c;
    st->sn[j] = s;
    col[j] = r;
    col[j + 1] = mk(0.0, 0.0);
    const cd gnext = -(conjc(s) * sc.gj);
    st->g[j + 1] = gnext;
    st->g[j] = c * sc.gj;
    double est = sqrt(abs2(gnext)) / sc.bnorm;
    st->est = est;
    if (sc.its < KMAXIT) st->hist[sc.its] = est;
    st->its = sc.its + 1;
    st->kcols = j + 1;
    bool fin = isfinite(est) && isfinite(hn);
    if (!fin) st->nonfinite = 1;
    st->done = (est <= tol || !fin || hn == 0.0 || cancel || sc.its + 1 >= sc.maxit) ? 1 : 0;
  }
  __syncthreads();
  for (int i = t; i <= j + 1; i += 64) st->H[i + ld * j] = L.col[i];
  if (t <= j) st->c[t] = L.sc[t];
}

// the column's finish as a launch of its own (one wavefront), after k_fin_sum
__global__ void __launch_bounds__(64) k_givens(KrylovArgs a, int j, double tol) {
  __shared__ GivensLds L;
  KrylovState* st = at_rhs(a).st;
  if (st->done) return;            // converged in an earlier column: the state stays as it is
  GivensScal sc;
  givens_stage(L, st, j, sc);
  givens_finish(L, a, st, j, tol, sc);
}

// one block per value: st->h1[i] = sum over the dot pass's blocks of part[i]; the block
// that stores the last of the 2 j + 3 sums of its right-hand side (a device-scope ticket,
// returned to zero by that block) then finishes the column (givens_finish).  The sums are
// formed in a fixed order whichever block finishes last.  Every block stages the column's
// inputs from earlier launches before its ticket, so that their loads overlap the fences.
__global__ void __launch_bounds__(256) k_fin_givens(KrylovArgs a, int j, double tol) {
  __shared__ cd lds[4];
  __shared__ int last;
  __shared__ GivensLds L;
  const RhsPtr p = at_rhs(a);
  KrylovState* st = p.st;
  const int i = blockIdx.x;
  const bool live = !st->done;         // converged in an earlier column: the state stays as it is
  cd v = mk(0.0, 0.0);
  v = sum_strided(p.part + (long long)i * a.pcap, a.nblk);
  block_sum(v, lds, st->h1 + i);
  GivensScal sc;
  if (live) givens_stage(L, st, j, sc);
  if (threadIdx.x == 0) {
    __threadfence();                     // this block's sum before its ticket
    last = atomicAdd(&st->ticket, 1) == (int)gridDim.x - 1;
    if (last) {
      __threadfence();                   // every other block's sum after their tickets
      st->ticket = 0;
    }
  }
  __syncthreads();
  if (!last) return;
  if (live) givens_finish(L, a, st, j, tol, sc);
}


// V_{j+1} = (H z_j - sum_i c_i V_i) / h_{j+1,j}.  The blocks take the nodes in reverse
// order, so that the first nodes they read are the last the dots pass read.  This pass is
// the basis's last reader in the iteration: its loads are non-temporal, so that they do
// not displace the data the next iteration's cycle reuses (the coarsest factors, the
// level-2 coefficients).
// With pack_dst, the first block of each right-hand side also packs its state (final after
// the column's finish) into the host-mapped slot, so that the stores to host memory drain
// while this pass streams instead of delaying it; the host reads the slot after an event
// recorded behind the launch, whose completion makes them visible (no fence of system scope).
template <typename CZ, int CMP>
__global__ void __launch_bounds__(256) k_arnoldi_update(KrylovArgs a, const CZ* __restrict__ z, int j,
                                                        char* pack_dst) {
  __shared__ cd sc[KMAXM + 1];
  __shared__ double sinv;
  const RhsPtr p = at_rhs(a);
  if (pack_dst && blockIdx.x == 0) pack_state(p.st, pack_dst, blockIdx.y);
  z += blockIdx.y * a.op.g.tot;
  if (p.st->done) return;
  if (threadIdx.x <= j) sc[threadIdx.x] = p.st->c[threadIdx.x];
  if (threadIdx.x == 0) sinv = p.st->hnext > 0.0 ? 1.0 / p.st->hnext : 0.0;
  const long long N = a.op.g.tot;
  const long long blk = (long long)gridDim.x - 1 - blockIdx.x;
  long long f[KNPT];
  bool ok[KNPT];
  for (int q = 0; q < KNPT; ++q) {
    long long t = (blk * KNPT + q) * 256 + threadIdx.x;
    ok[q] = t < N;
    f[q] = ok[q] ? t : N - 1;
  }
  cd w[KNPT], nx[KNPT];
  for (int q = 0; q < KNPT; ++q) nx[q] = ld_nt(p.V + f[q]);
  for (int q = 0; q < KNPT; ++q) w[q] = apply_h<CMP>(a, z, f[q]);
  __syncthreads();
  for (int i = 0; i <= j; ++i) {
    cd vi[KNPT];
    for (int q = 0; q < KNPT; ++q) vi[q] = nx[q];
    const long long in = (long long)(i < j ? i + 1 : j) * a.ldv;   // the last pass reloads V_j
    for (int q = 0; q < KNPT; ++q) nx[q] = ld_nt(p.V + in + f[q]);
    const cd ci = sc[i];
    for (int q = 0; q < KNPT; ++q) w[q] -= ci * vi[q];
  }
  const double si = sinv;
  for (int q = 0; q < KNPT; ++q)
    if (ok[q]) p.V[(long long)(j + 1) * a.ldv + f[q]] = si * w[q];
}

// restart bookkeeping from tmp = (||r||^2, ||b||^2): beta0, g = beta0 e1
__global__ void k_fin_residual(KrylovArgs a, int set_b) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const RhsPtr p = at_rhs(a);
  KrylovState* st = p.st;
  if (set_b) st->bnorm = sqrt(st->tmp[0].y);
  double b0 = sqrt(st->tmp[0].x);
  st->beta0 = b0;
  st->g[0] = mk(b0, 0.0);
  for (int i = 1; i <= KMAXM; ++i) st->g[i] = mk(0.0, 0.0);
  st->true_rel = st->bnorm > 0.0 ? b0 / st->bnorm : 0.0;
  st->done = st->final;
  st->kcols = 0;
  if (!isfinite(b0)) st->nonfinite = 1;
}

__global__ void __launch_bounds__(256) k_scale_v0(KrylovArgs a) {
  const RhsPtr p = at_rhs(a);
  double s = p.st->beta0 > 0.0 ? 1.0 / p.st->beta0 : 0.0;
  const long long N = a.op.g.tot;
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f < N) p.V[f] = s * p.V[f];
  }
}

// y = R^{-1} g on the k x k upper triangle of the rotated Hessenberg matrix (k: the
// columns of the current cycle)
__global__ void k_solve_y(KrylovArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const RhsPtr p = at_rhs(a);
  KrylovState* st = p.st;
  const int k = st->nonfinite ? 0 : st->kcols;     // a non-finite column leaves x as it is
  const int ld = KMAXM + 1;
  for (int i = k - 1; i >= 0; --i) {
    cd acc = st->g[i];
    for (int l = i + 1; l < k; ++l) acc -= st->H[i + ld * l] * st->y[l];
    st->y[i] = cdiv(acc, st->H[i + ld * i]);
  }
}

// x += sum_i y_i Z_i
template <typename CZ>
__global__ void __launch_bounds__(256) k_update_x(KrylovArgs a, const CZ* __restrict__ Z, long long ldz,
                                                  cd* __restrict__ x) {
  __shared__ cd sy[KMAXM];
  const RhsPtr p = at_rhs(a);
  Z += blockIdx.y * a.op.g.tot;
  x += blockIdx.y * a.op.g.tot;
  const int k = p.st->nonfinite ? 0 : p.st->kcols;
  if (threadIdx.x < k) sy[threadIdx.x] = p.st->y[threadIdx.x];
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

// x += z over nr right-hand sides (z in cycle precision)
template <typename CZ>
__global__ void __launch_bounds__(256) k_add_z(KrylovArgs a, const CZ* __restrict__ z, cd* __restrict__ x) {
  const long long N = a.op.g.tot;
  z += blockIdx.y * N;
  x += blockIdx.y * N;
  for (int q = 0; q < KNPT; ++q) {
    long long f = node_of(q);
    if (f < N) x[f] += to_d(z[f]);
  }
}

__global__ void k_zero_c128(cd* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = mk(0.0, 0.0);
}

__global__ void k_init_state(KrylovState* st, int maxit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st += blockIdx.y;
    st->its = 0;
    st->nonfinite = 0;
    st->done = 0;
    st->final = 0;
    st->kcols = 0;
    st->maxit = maxit;
    st->ticket = 0;
  }
}

// the scalar blocks (bnorm .. hist) of the nrhs states, packed one after the other into
// host-visible memory (pinned, written through), for the host to read after an event
// (the host reads dst after synchronising with the stream or an event behind this launch,
// which makes the stores visible: no fence of system scope)
__global__ void k_pack_states(const KrylovState* st, char* dst, int nrhs) {
  for (int r = 0; r < nrhs; ++r) pack_state(st + r, dst, r);
}

// right-hand sides in mask: finished, done from now on
__global__ void k_finalize(KrylovState* st, unsigned mask) {
  if (threadIdx.x == 0 && ((mask >> blockIdx.y) & 1u)) {
    st[blockIdx.y].done = 1;
    st[blockIdx.y].final = 1;
  }
}

// timing runs only: keeps the stream busy for about rounds x 3.4 us (s_sleep 127 = 8128
// clocks) so that the host has queued the launches that follow, with their timing events,
// before the device reaches them; the event pairs then time the kernels, not host gaps
__global__ void k_hold(int rounds) {
  for (int i = 0; i < rounds; ++i) __builtin_amdgcn_s_sleep(127);
}

// ------------------------------------------------------------- launchers ----
void kr_hold(int rounds, hipStream_t s) { hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, s, rounds); }
void kr_pack_states(const KrylovArgs& a, void* host_dst, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_states, dim3(1), dim3(256), 0, s, a.st, (char*)host_dst, a.nrhs);
}
void kr_finalize(const KrylovArgs& a, unsigned mask, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1, a.nrhs), dim3(1), 0, s, a.st, mask);
}
void kr_init(const KrylovArgs& a, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1, a.nrhs), dim3(1), 0, s, a.st, max_iter);
}
void kr_residual(const KrylovArgs& a, const cd* x, const cd* b, int with_b, hipStream_t s) {
  if (a.op.compact)
    hipLaunchKernelGGL((k_residual<1>), dim3(a.nblk, a.nrhs), dim3(256), 0, s, a, x, b);
  else
    hipLaunchKernelGGL((k_residual<0>), dim3(a.nblk, a.nrhs), dim3(256), 0, s, a, x, b);
  hipLaunchKernelGGL(k_fin_sum, dim3(1, a.nrhs), dim3(256), 0, s, a, offsetof(KrylovState, tmp));
  hipLaunchKernelGGL(k_fin_residual, dim3(1, a.nrhs), dim3(1), 0, s, a, with_b);
}
void kr_scale_v0(const KrylovArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_v0, dim3(a.nblk, a.nrhs), dim3(256), 0, s, a);
}
void kr_arnoldi(const KrylovArgs& a, const void* z, int z_f32, int j, double tol, void* pack_dst, int fused,
                hipStream_t s) {
  dim3 g(a.nblk, a.nrhs);
  const int cmp = a.op.compact;
  if (z_f32 && !cmp)
    hipLaunchKernelGGL((k_arnoldi_dots<cf, 0>), g, dim3(256), 0, s, a, (const cf*)z, j);
  else if (!cmp)
    hipLaunchKernelGGL((k_arnoldi_dots<cd, 0>), g, dim3(256), 0, s, a, (const cd*)z, j);
  else if (z_f32)
    hipLaunchKernelGGL((k_arnoldi_dots<cf, 1>), g, dim3(256), 0, s, a, (const cf*)z, j);
  else
    hipLaunchKernelGGL((k_arnoldi_dots<cd, 1>), g, dim3(256), 0, s, a, (const cd*)z, j);
  if (fused) {
    hipLaunchKernelGGL(k_fin_givens, dim3(2 * j + 3, a.nrhs), dim3(256), 0, s, a, j, tol);
  } else {
    hipLaunchKernelGGL(k_fin_sum, dim3(2 * j + 3, a.nrhs), dim3(256), 0, s, a, offsetof(KrylovState, h1));
    hipLaunchKernelGGL(k_givens, dim3(1, a.nrhs), dim3(64), 0, s, a, j, tol);
  }
  char* pk = (char*)pack_dst;
  if (z_f32 && !cmp)
    hipLaunchKernelGGL((k_arnoldi_update<cf, 0>), g, dim3(256), 0, s, a, (const cf*)z, j, pk);
  else if (!cmp)
    hipLaunchKernelGGL((k_arnoldi_update<cd, 0>), g, dim3(256), 0, s, a, (const cd*)z, j, pk);
  else if (z_f32)
    hipLaunchKernelGGL((k_arnoldi_update<cf, 1>), g, dim3(256), 0, s, a, (const cf*)z, j, pk);
  else
    hipLaunchKernelGGL((k_arnoldi_update<cd, 1>), g, dim3(256), 0, s, a, (const cd*)z, j, pk);
}
void kr_update_x(const KrylovArgs& a, const void* Z, int z_f32, long long ldz, cd* x, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_y, dim3(1, a.nrhs), dim3(1), 0, s, a);
  dim3 g(a.nblk, a.nrhs);
  if (z_f32)
    hipLaunchKernelGGL((k_update_x<cf>), g, dim3(256), 0, s, a, (const cf*)Z, ldz, x);
  else
    hipLaunchKernelGGL((k_update_x<cd>), g, dim3(256), 0, s, a, (const cd*)Z, ldz, x);
}
void kr_add_z(const KrylovArgs& a, const void* z, int z_f32, cd* x, hipStream_t s) {
  dim3 g(a.nblk, a.nrhs);
  if (z_f32)
    hipLaunchKernelGGL((k_add_z<cf>), g, dim3(256), 0, s, a, (const cf*)z, x);
  else
    hipLaunchKernelGGL((k_add_z<cd>), g, dim3(256), 0, s, a, (const cd*)z, x);
}
void kr_zero(cd* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_c128, dim3(1024), dim3(256), 0, s, x, n);
}

}  // namespace helm
