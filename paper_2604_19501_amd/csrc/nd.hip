// Exact solve of the real-shifted coarsest operator A3 (eq. 3.6) on the GPU.
//
// Factorisation (setup, FP64): fronts are processed by height in the nested-
// dissection tree (nd_plan.cpp).  A front matrix F (nF x nF, S nodes first) is
// assembled from the original coefficients and the children's Schur complements
// (extend-add), then its S pivots are exchanged by Gauss-Jordan steps with
// partial pivoting among the S rows.  The exchange of a pivot set K turns the
// relation y = F x into [x_S; y_B] = F' [y_S; x_B]:
//     F'_SS = A^-1,   F'_SB = -A^-1 B,   F'_BS = C A^-1,   F'_BB = D - C A^-1 B,
// with A = F_SS, B = F_SB, C = F_BS, D = F_BB.  Pivots are taken in panels of
// kb columns: within a panel the exchange updates only the panel columns; the
// other columns then get one rank-kb update  F[:, J] = F0[:, J] - F'[:, K] F[K, J]
// (rows K of F0 zeroed), a GEMM.  Row interchanges permute equations only, so
// the columns of the left block are un-permuted at the end.
//
// Solve (per right-hand side, cycle precision): forward over the tree bottom-up,
//     [g_S; t_B] = [A^-1; C A^-1] f_S,   u_B = v_B - t_B  (passed to the parent),
// then backward top-down,  x_S = g_S + (-A^-1 B) x_B.
#include <stdexcept>

#include "internal.h"

namespace helm {

// ----------------------------------------------------------------- setup ----
__global__ void k_zero_d2(cd* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = mk(0.0, 0.0);
}

__global__ void __launch_bounds__(256) k_nd_assemble(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                     const NDAsm* __restrict__ asmv, const cd* __restrict__ coef,
                                                     cd* __restrict__ Fp) {
  const NDFrontDev f = fr[ids[blockIdx.y]];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < f.asm_cnt;
       e += (long long)gridDim.x * blockDim.x) {
    NDAsm a = asmv[f.asm_off + e];
    cd* F = Fp + f.F_off;
    F[(long long)a.row * f.nF + a.col] += coef[a.cidx];
  }
}

// the front record of work slot y: with ids, fr is the plan's array; without, fr already
// holds the fronts of one height in slot order (one load instead of two dependent ones)
__device__ __forceinline__ NDFrontDev front_at(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids, int y) {
  return ids ? fr[ids[y]] : fr[y];
}

__global__ void __launch_bounds__(256) k_nd_extend(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                   const int* __restrict__ children,
                                                   const long long* __restrict__ child_map_off,
                                                   const int* __restrict__ maps, cd* __restrict__ Fp, int slot) {
  const NDFrontDev f = fr[ids[blockIdx.y]];
  if (slot >= f.nchild) return;
  const NDFrontDev fc = fr[children[f.child_off + slot]];
  long long n2 = (long long)fc.nB * fc.nB;
  const int* mp = maps + child_map_off[f.child_off + slot];
  cd* F = Fp + f.F_off;
  const cd* Fc = Fp + fc.F_off;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n2; p += (long long)gridDim.x * blockDim.x) {
    int k1 = (int)(p / fc.nB), k2 = (int)(p % fc.nB);
    F[(long long)mp[k1] * f.nF + mp[k2]] += Fc[(long long)(fc.nS + k1) * fc.nF + fc.nS + k2];
  }
}

// Panel [k0, k0 + kbb) of every front of one height with the panel block held in
// registers: one NT-thread work-group per front, thread t owning rows t, t + NT, ...
// (R rows of KB entries each, and the rows' permutation entries).  Per pivot: a
// block-wide argmax (the candidates come out of the previous pivot's update), the
// exchange of rows k and p through LDS (the new pivot row is then read by every thread),
// and the exchange update of each owned row in registers.  Row swaps of the columns
// outside the panel are recorded in swp and applied by k_nd_swap_rest.
// (v, i) <- the larger value, the lower index on ties; branch-free
__device__ __forceinline__ void amax_step(double& v, int& i, double ov, int oi) {
  const bool t = (ov > v) | ((ov == v) & (oi < i));
  v = t ? ov : v;
  i = t ? oi : i;
}

// one argmax step against the lane chosen by a DPP permutation (quad_perm / mirrors)
template <int CTRL>
__device__ __forceinline__ void amax_dpp(double& v, int& i) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  const int oi = __builtin_amdgcn_mov_dpp(i, CTRL, 0xf, 0xf, false);
  amax_step(v, i, __hiloint2double(hi, lo), oi);
}

// argmax over the 16 lanes of each DPP row: xor 1, xor 2 (quad permutations), then the
// half-row and row mirrors; every lane of a row ends with the row's result
__device__ __forceinline__ void amax_row16(double& v, int& i) {
  amax_dpp<0xB1>(v, i);
  amax_dpp<0x4E>(v, i);
  amax_dpp<0x141>(v, i);
  amax_dpp<0x140>(v, i);
}

__device__ __forceinline__ void amax_lane(double& v, int& i, double w, int j, int lane) {
  amax_step(v, i, __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(w), lane),
                                   __builtin_amdgcn_readlane(__double2loint(w), lane)),
            __builtin_amdgcn_readlane(j, lane));
}

// block-wide argmax (at most 16 waves); the result is uniform.  sv / si may be rewritten
// only after a later barrier.
__device__ __forceinline__ void argmax_block(double v, int idx, double* sv, int* si, double& bv, int& bi) {
  amax_row16(v, idx);
  double w = v;
  int j = idx;
  v = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(w), 0), __builtin_amdgcn_readlane(__double2loint(w), 0));
  idx = __builtin_amdgcn_readlane(j, 0);
  amax_lane(v, idx, w, j, 16);
  amax_lane(v, idx, w, j, 32);
  amax_lane(v, idx, w, j, 48);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  if (lane == 0) { sv[wv] = v; si[wv] = idx; }
  __syncthreads();
  v = lane < nw ? sv[lane] : -2.0;
  idx = lane < nw ? si[lane] : 0x7fffffff;
  amax_row16(v, idx);
  bv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0), __builtin_amdgcn_readlane(__double2loint(v), 0));
  bi = __builtin_amdgcn_readlane(idx, 0);
}

// panel width of the register panel for fronts of up to nF rows (0: too large for it)
int panel_reg_kb(int nF) { return nF <= 256 ? 32 : nF <= 1024 ? 16 : nF <= 2048 ? 8 : 0; }

// The column loop stays rolled (an unrolled one overflows the instruction cache); so that
// registers are still indexed by constants, a thread's KB entries of a row are kept
// rotated: before pivot kk, slot jj holds panel column (kk + jj) mod KB, the update of
// pivot kk writes column (kk + 1 + jj) mod KB into slot jj.
template <int KB, int R, int NT>
__global__ void __launch_bounds__(NT) k_nd_panel_reg(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                     cd* __restrict__ Fp, int* __restrict__ perm,
                                                     int* __restrict__ swp, int k0, int* __restrict__ err) {
  __shared__ cd s_rk[KB], s_rp[KB];      // rows p (the new pivot row k) and k before the swap, by column
  __shared__ int s_pp, s_pk;              // their permutation entries
  __shared__ double s_v[16];
  __shared__ int s_i[16];
  const NDFrontDev f = front_at(fr, ids, blockIdx.x);
  if (f.nS <= k0) return;
  const int kbb = min(KB, f.nS - k0);
  const int nF = f.nF, nS = f.nS, tid = threadIdx.x, w0 = tid & ~63;
  cd* F = Fp + f.F_off;
  int* pm = perm + f.perm_off;
  int* sw = swp + (long long)blockIdx.x * ND_KBMAX;
  cd a[R][KB];
  int pr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = min(tid + r * NT, nF - 1);
    const long long row = (long long)i * nF + k0;
#pragma unroll
    for (int jj = 0; jj < KB; ++jj) a[r][jj] = F[row + min(jj, kbb - 1)];
    pr[r] = pm[min(i, nS - 1)];
  }
  double best = -1.0;
  int bi = k0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + r * NT;
    if (i >= k0 && i < nS) amax_step(best, bi, abs2(a[r][0]), i);
  }
  for (int kk = 0; kk < kbb; ++kk) {
    const int k = k0 + kk;
    double pv;
    int p;
    argmax_block(best, bi, s_v, s_i, pv, p);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + r * NT;
      if (i == p) {
#pragma unroll
        for (int jj = 0; jj < KB; ++jj) s_rk[(kk + jj) % KB] = a[r][jj];
        s_pp = pr[r];
      }
      if (i == k) {
#pragma unroll
        for (int jj = 0; jj < KB; ++jj) s_rp[(kk + jj) % KB] = a[r][jj];
        s_pk = pr[r];
      }
    }
    if (tid == 0) {
      sw[kk] = p;
      if (!(pv > 0.0)) atomicOr(err, 1);
    }
    __syncthreads();
    cd piv = s_rk[kk];
    if (!(pv > 0.0)) piv = mk(1.0, 0.0);
    const cd inv = cdiv(mk(1.0, 0.0), piv);
    best = -1.0;
    bi = k + 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (w0 + r * NT >= nF) continue;           // the wave's rows of this slot are all padding
      const int i = tid + r * NT;
      if (i == p && p != k) {                    // row p takes the old row k
#pragma unroll
        for (int jj = 0; jj < KB; ++jj) a[r][jj] = s_rp[(kk + jj) % KB];
        pr[r] = s_pk;
      }
      if (i == k) {                              // the pivot row after the exchange
#pragma unroll
        for (int jj = 0; jj + 1 < KB; ++jj) a[r][jj] = -(s_rk[(kk + 1 + jj) % KB] * inv);
        a[r][KB - 1] = inv;
        pr[r] = s_pp;
      } else {                                   // exchange update, shifted by one slot
        const cd ck = a[r][0] * inv;
#pragma unroll
        for (int jj = 0; jj + 1 < KB; ++jj) a[r][jj] = a[r][jj + 1] - ck * s_rk[(kk + 1 + jj) % KB];
        a[r][KB - 1] = ck;
        if (kk + 1 < kbb && i > k && i < nS) amax_step(best, bi, abs2(a[r][0]), i);
      }
    }
  }
  // slot jj now holds column (kbb + jj) mod KB
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + r * NT;
    if (i < nF)
#pragma unroll
      for (int jj = 0; jj < KB; ++jj) {
        const int c = (kbb + jj) % KB;
        if (c < kbb) F[(long long)i * nF + k0 + c] = a[r][jj];
      }
    if (i >= k0 && i < nS) pm[i] = pr[r];
  }
}

// Panel [k0, k0 + kbb) of fronts too large for an LDS-resident panel: every pivot step
// is spread over work-groups of PROWS rows.
//   k_piv_search   argmax of |F[i][k0]| over the S rows i >= k0 of each row block
//   k_piv_step     one launch per pivot: the pivot from the block candidates, the exchange
//                  of its row block from one panel copy into the other, and the block's
//                  candidate for the next column; the swap of the other columns is
//                  recorded (k_nd_swap_rest)
//   k_piv_back     the panel copied back into the front where its column count is odd
// Arithmetic and pivot choice are those of the single-work-group exchange, so the
// factors do not depend on which path a front takes.
#define PROWS 32
__device__ __forceinline__ void cand_argmax(double v, int i, double* sv, int* si, int nt) {
  // block-wide (nt threads) argmax with the lower index on ties; result in sv[0], si[0]
  for (int o = 32; o > 0; o >>= 1) {
    double ov = __shfl_xor(v, o, 64);
    int oi = __shfl_xor(i, o, 64);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { sv[w] = v; si[w] = i; }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 1; q < nt / 64; ++q)
      if (sv[q] > sv[0] || (sv[q] == sv[0] && si[q] < si[0])) { sv[0] = sv[q]; si[0] = si[q]; }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_piv_search(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                    const cd* __restrict__ Fp, int k, PivCand* __restrict__ cand,
                                                    int nblk) {
  __shared__ double sv[4];
  __shared__ int si[4];
  const NDFrontDev f = front_at(fr, ids, blockIdx.y);
  if (f.nS <= k || (int)blockIdx.x * PROWS >= f.nF) return;
  const cd* F = Fp + f.F_off;
  double best = -1.0;
  int bi = 0x7fffffff;
  const int r0 = max(k, (int)blockIdx.x * PROWS), r1 = min(f.nS, ((int)blockIdx.x + 1) * PROWS);
  for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
    double v = abs2(F[(long long)i * f.nF + k]);
    if (v > best) { best = v; bi = i; }
  }
  cand_argmax(best, bi, sv, si, blockDim.x);
  if (threadIdx.x == 0) cand[(long long)blockIdx.y * nblk + blockIdx.x] = PivCand{sv[0], si[0], 0};
}

// One pivot step of a multi-work-group panel in one launch.  Every work-group reduces the
// row blocks' candidates to the pivot p exactly as a single reduction would (the larger
// value, the lower row on ties), reads the pivot row, and writes the exchange update of its
// rows from the panel copy S into the other copy D: the front itself and a panel buffer
// alternate by column, so no work-group reads what another writes in the same launch, and
// rows k and p are read exchanged instead of being swapped in place.  The front's first
// work-group records the swap and the permutation.  The arithmetic is that of the
// single-work-group exchange, so the factors do not depend on the path a front takes.
template <int CW>
__global__ void __launch_bounds__(256) k_piv_step(const NDFrontDev* __restrict__ fr, cd* __restrict__ Fp,
                                                  cd* __restrict__ Pb, long long pstride, int s_is_pb, int k0, int kb,
                                                  int kk, const PivCand* __restrict__ cin, PivCand* __restrict__ cout,
                                                  int nblk, int* __restrict__ perm, int* __restrict__ swp,
                                                  int* __restrict__ err) {
  constexpr int RPP = 256 / CW, NP = PROWS / RPP;
  __shared__ cd srk[ND_KBMAX];
  __shared__ double sv[4];
  __shared__ int si[4];
  const NDFrontDev f = fr[blockIdx.y];
  const int k = k0 + kk;
  if (f.nS <= k || (int)blockIdx.x * PROWS >= f.nF) return;
  const int kbb = min(kb, f.nS - k0);
  // row i of the panel: F + F_off + i nF + k0 in the front, Pb + y pstride + i kb in the buffer
  cd* const Fr = Fp + f.F_off + k0;
  cd* const Pr = Pb + (long long)blockIdx.y * pstride;
  const cd* const S = s_is_pb ? Pr : Fr;
  cd* const D = s_is_pb ? Fr : Pr;
  const long long lS = s_is_pb ? kb : f.nF, lD = s_is_pb ? f.nF : kb;
  const int t = threadIdx.x;
  const int jj = t & (CW - 1), rsub = t / CW;
  const int r0 = (int)blockIdx.x * PROWS + rsub;
  const int jl = min(jj, kbb - 1);
  // the block's rows as they stand (rows k and p are read again below, exchanged): these
  // loads do not depend on the pivot and overlap its reduction
  cd ckv[NP], rv[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const long long i = min(r0 + RPP * q, f.nF - 1);
    ckv[q] = S[i * lS + kk];
    rv[q] = S[i * lS + jl];
  }
  double best = -1.0;
  int bi = 0x7fffffff;
  const int nb = (f.nF + PROWS - 1) / PROWS;
  for (int b = t + k / PROWS; b < nb && b * PROWS < f.nS; b += 256) {
    const PivCand c = cin[(long long)blockIdx.y * nblk + b];
    if (c.v > best || (c.v == best && c.i < bi)) {
      best = c.v;
      bi = c.i;
    }
  }
  cand_argmax(best, bi, sv, si, blockDim.x);
  const double pv = sv[0];
  const int p = pv >= 0.0 && si[0] < f.nS ? si[0] : k;
  if (t < kbb) srk[t] = S[(long long)p * lS + t];      // the pivot row: old row p
  if (blockIdx.x == 0 && t == 0) {
    swp[(long long)blockIdx.y * ND_KBMAX + kk] = p;
    if (p != k) {
      const int q = perm[f.perm_off + k];
      perm[f.perm_off + k] = perm[f.perm_off + p];
      perm[f.perm_off + p] = q;
    }
    if (!(pv > 0.0)) atomicOr(err, 1);
  }
  // rows k and p of this block take each other's content
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int i = r0 + RPP * q;
    if (p != k && i < f.nF && (i == k || i == p)) {
      const long long src = i == k ? p : k;
      ckv[q] = S[src * lS + kk];
      rv[q] = S[src * lS + jl];
    }
  }
  __syncthreads();
  cd piv = srk[kk];
  if (!(pv > 0.0)) piv = mk(1.0, 0.0);
  const cd inv = cdiv(mk(1.0, 0.0), piv);
  const bool next = kk + 1 < kbb;
  best = -1.0;
  bi = 0x7fffffff;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int i = r0 + RPP * q;
    if (i >= f.nF) continue;
    cd* row = D + (long long)i * lD;
    if (i == k) {
      if (jj < kbb) row[jj] = jj == kk ? inv : -(srk[jj] * inv);
      continue;
    }
    const cd ck = ckv[q] * inv;
    cd nv = mk(0.0, 0.0);
    if (jj < kbb) {
      nv = jj == kk ? ck : rv[q] - ck * srk[jj];
      row[jj] = nv;
    }
    if (next && jj == kk + 1 && i > k && i < f.nS) {
      double v = abs2(nv);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
  }
  if (next) {
    cand_argmax(best, bi, sv, si, blockDim.x);
    if (t == 0) cout[(long long)blockIdx.y * nblk + blockIdx.x] = PivCand{sv[0], si[0], 0};
  }
}

// fronts whose panel has an odd column count end in the buffer: copy it back
__global__ void __launch_bounds__(256) k_piv_back(const NDFrontDev* __restrict__ fr, cd* __restrict__ Fp,
                                                  const cd* __restrict__ Pb, long long pstride, int k0, int kb) {
  const NDFrontDev f = fr[blockIdx.y];
  if (f.nS <= k0) return;
  const int kbb = min(kb, f.nS - k0);
  if ((kbb & 1) == 0) return;
  const int r = (int)blockIdx.x * PROWS + (int)threadIdx.x / 8;
  if (r >= f.nF) return;
  const cd* src = Pb + (long long)blockIdx.y * pstride + (long long)r * kb;
  cd* dst = Fp + f.F_off + (long long)r * f.nF + k0;
  for (int j = threadIdx.x % 8; j < kbb; j += 8) dst[j] = src[j];
}

// apply the panel's recorded row swaps to the columns outside the panel
__global__ void __launch_bounds__(256) k_nd_swap_rest(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                      cd* __restrict__ Fp, const int* __restrict__ swp, int k0,
                                                      int KB) {
  const NDFrontDev f = front_at(fr, ids, blockIdx.y);
  if (f.nS <= k0) return;
  const int kbb = min(KB, f.nS - k0);
  const int* sw = swp + (long long)blockIdx.y * ND_KBMAX;
  cd* F = Fp + f.F_off;
  for (int jj = blockIdx.x * blockDim.x + threadIdx.x; jj < f.nF - kbb; jj += gridDim.x * blockDim.x) {
    int j = jj < k0 ? jj : jj + kbb;
    for (int kk = 0; kk < kbb; ++kk) {
      int p = sw[kk], k = k0 + kk;
      if (p != k) {
        cd t = F[(long long)k * f.nF + j];
        F[(long long)k * f.nF + j] = F[(long long)p * f.nF + j];
        F[(long long)p * f.nF + j] = t;
      }
    }
  }
}

// Columns J of an exchange update: the front's columns [lo, hi) without the pivot block
// K = [k0, k0 + kbb).  un < 0: [lo, hi) = [0, nF), the trailing update of every other
// column; otherwise [u0, min(u0 + un, nS)), the other panels of one column block, which
// the block's pivots reach before the trailing update does.
struct ColMap {
  int lo, k0, kbb, ncol;
  __device__ __forceinline__ int col(int c) const {
    const int j = lo + c;
    return j >= k0 ? j + kbb : j;
  }
};
__device__ __forceinline__ bool col_map(const NDFrontDev& f, int k0, int kb, int u0, int un, ColMap& m) {
  m.kbb = min(kb, f.nS - k0);
  if (m.kbb <= 0) return false;
  m.lo = un < 0 ? 0 : u0;
  const int hi = un < 0 ? f.nF : min(u0 + un, f.nS);
  m.k0 = k0;
  m.ncol = hi - m.lo - m.kbb;
  return m.ncol > 0;
}

// T = F[K rows][J columns], then zero those entries
__global__ void __launch_bounds__(256) k_nd_save_t(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                   const long long* __restrict__ toff, cd* __restrict__ Fp,
                                                   cd* __restrict__ T, int k0, int kb, int u0, int un) {
  const NDFrontDev f = front_at(fr, ids, blockIdx.y);
  ColMap cm;
  if (!col_map(f, k0, kb, u0, un, cm)) return;
  const int ncol = cm.ncol;
  cd* F = Fp + f.F_off;
  cd* Tt = T + toff[blockIdx.y];
  long long n = (long long)cm.kbb * ncol;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
    int kk = (int)(p / ncol), jj = (int)(p % ncol);
    long long a = (long long)(k0 + kk) * f.nF + cm.col(jj);
    Tt[p] = F[a];
    F[a] = mk(0.0, 0.0);
  }
}

// F[:, J] -= F[:, K] * T  (complex FP64 GEMM on the matrix cores).  A work-group owns a
// 64 x 64 tile of C = F[:, J]; each wavefront a 32 x 32 quarter as 2 x 2 blocks of the
// 16 x 16 x 4 FP64 MFMA, real and imaginary parts accumulated separately:
//   Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br  (four real MFMAs per k group).
// MFMA lane layout: A[m][k] from lane m + 16 k, B[k][n] from lane n + 16 k, and lane l
// holds D[l / 16 + 4 i][l % 16], i < 4.  Panels of A and B pass through LDS, 16 k at a time.
#define GT 64
#define GK 16
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) k_nd_gemm(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                 const long long* __restrict__ toff, cd* __restrict__ Fp,
                                                 const cd* __restrict__ T, int k0, int kb, int u0, int un) {
  const NDFrontDev f = front_at(fr, ids, blockIdx.y);
  ColMap cm;
  if (!col_map(f, k0, kb, u0, un, cm)) return;
  const int kbb = cm.kbb;
  const int M = f.nF, Ncol = cm.ncol;
  const int tilesN = (Ncol + GT - 1) / GT, tilesM = (M + GT - 1) / GT;
  if ((int)blockIdx.x >= tilesM * tilesN) return;
  const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;
  cd* F = Fp + f.F_off;
  const cd* Tt = T + toff[blockIdx.y];
  __shared__ cd sA[GK][GT + 1];
  __shared__ cd sB[GK][GT + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;       // wavefront's quarter of the tile
  mfma_d4 accr[2][2], acci[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = mfma_d4{0.0, 0.0, 0.0, 0.0};
      acci[a][b] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    }
  const int lm = lane & 15, lk = lane >> 4;
  // the next k slice is loaded into registers while the matrix cores work on this one
  constexpr int NLD = GK * GT / 256;
  cd ra[NLD], rb[NLD];
  auto load = [&](int kk0) {
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
      const int p = (int)threadIdx.x + 256 * it;
      const int kk = p % GK, r = p / GK;             // A tile: consecutive threads along a row
      const int row = tm * GT + r, kq = kk0 + kk;
      ra[it] = (row < M && kq < kbb) ? F[(long long)row * f.nF + k0 + kq] : mk(0.0, 0.0);
      const int kk2 = p / GT, c = p % GT;            // B tile: consecutive threads along a row of T
      const int col = tn * GT + c, kq2 = kk0 + kk2;
      rb[it] = (col < Ncol && kq2 < kbb) ? Tt[(long long)kq2 * Ncol + col] : mk(0.0, 0.0);
    }
  };
  load(0);
  for (int kk0 = 0; kk0 < kbb; kk0 += GK) {
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
      const int p = (int)threadIdx.x + 256 * it;
      sA[p % GK][p / GK] = ra[it];
      sB[p / GT][p % GT] = rb[it];
    }
    __syncthreads();
    if (kk0 + GK < kbb) load(kk0 + GK);
#pragma unroll
    for (int k4 = 0; k4 < GK; k4 += 4) {
      cd av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = sA[k4 + lk][wr + 16 * q + lm];
        bv[q] = sB[k4 + lk][wc + 16 * q + lm];
      }
      // the four products of a block go to two accumulators: issue them in rounds over the
      // eight accumulators, so that no MFMA waits for the one just before it
#pragma unroll
      for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
          accr[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[qa].x, bv[qb].x, accr[qa][qb], 0, 0, 0);
          acci[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[qa].x, bv[qb].y, acci[qa][qb], 0, 0, 0);
        }
#pragma unroll
      for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
          accr[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[qa].y, bv[qb].y, accr[qa][qb], 0, 0, 0);
          acci[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[qa].y, bv[qb].x, acci[qa][qb], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int qa = 0; qa < 2; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = tm * GT + wr + 16 * qa + lk + 4 * i;
        const int col = tn * GT + wc + 16 * qb + lm;
        if (row >= M || col >= Ncol) continue;
        cd* c = F + (long long)row * f.nF + cm.col(col);
        *c -= mk(accr[qa][qb][i], acci[qa][qb][i]);
      }
}

template <typename C>
__global__ void __launch_bounds__(256) k_nd_finalize(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                     const cd* __restrict__ Fp, const int* __restrict__ perm,
                                                     C* __restrict__ Lp, C* __restrict__ Wp) {
  const NDFrontDev f = front_at(fr, ids, blockIdx.y);
  const cd* F = Fp + f.F_off;
  const int* pm = perm + f.perm_off;
  long long nL = (long long)f.nF * f.nS, nW = (long long)f.nS * f.nB;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nL + nW;
       p += (long long)gridDim.x * blockDim.x) {
    if (p < nL) {                 // column pm[k] of L (column major, ld ldL) <- column k of F
      int i = (int)(p / f.nS), k = (int)(p % f.nS);
      Lp[f.L_off + (long long)pm[k] * f.ldL + i] = conv<C>::from(F[(long long)i * f.nF + k]);
    } else {                      // W (column major, ld ldW) <- F[0:nS, nS:nF]
      long long q = p - nL;
      int i = (int)(q / f.nB), j = (int)(q % f.nB);
      Wp[f.W_off + (long long)j * f.ldW + i] = conv<C>::from(F[(long long)i * f.nF + f.nS + j]);
    }
  }
}

__global__ void k_iota(int* __restrict__ p, const NDFrontDev* __restrict__ fr, int nfronts) {
  int t = blockIdx.x;
  if (t >= nfronts) return;
  const NDFrontDev f = fr[t];
  for (int i = threadIdx.x; i < f.nS; i += blockDim.x) p[f.perm_off + i] = i;
}

// ----------------------------------------------------------------- solve ----
template <typename C>
__device__ __forceinline__ C cmul_conj(C a, C x, int conj) {   // (conj? conj(a) : a) * x
  if (conj) a.y = -a.y;
  return a * x;
}


// one entry of a gather list: r at the row's node (rid >= 0), the first two updates inline
// and the rest through cidx; every load of the first level is issued unconditionally
template <typename C>
__device__ __forceinline__ C gather_list(const NDGather& g, const int* __restrict__ cidx, const C* __restrict__ upd,
                                         const C* __restrict__ r) {
  typedef decltype(r[0].x) R;
  const C a = r[max(g.rid, 0)], u0 = upd[max(g.u0, 0)], u1 = upd[max(g.u1, 0)];
  C v = g.rid >= 0 ? a : mk((R)0, (R)0);
  if (g.u0 >= 0) v += u0;
  if (g.u1 >= 0) v += u1;
  for (int q = g.ca; q < g.cb; ++q) v += upd[cidx[q]];
  return v;
}

// f_S (and v_B) entry i of front f: right-hand side on S plus the children's updates
// (contribution list cptr[i] .. cptr[i+1] of absolute indices into the update pool); F is
// the front record or a work item carrying its fields
template <typename C, typename F>
__device__ __forceinline__ C gather_entry(const F& f, const int* __restrict__ cptr,
                                          const int* __restrict__ cidx, const int* __restrict__ id,
                                          const C* __restrict__ upd, const C* __restrict__ r, int i) {
  typedef decltype(r[0].x) R;
  C v = i < f.nS ? r[id[i]] : mk((R)0, (R)0);
  const int* cp = cptr + f.inv_off;
  const int a = cp[i], b = cp[i + 1];
  for (int q = a; q < b; ++q) v += upd[cidx[q]];
  return v;
}

__device__ __forceinline__ size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }

// the five parts of a task's schedule copied to LDS in one pass: eight independent loads
// per thread and round before the stores (word w of the concatenation belongs to part r
// when end[r - 1] <= w < end[r])
struct LdsCopy5 {
  const int *s0, *s1, *s2, *s3, *s4;
  int *d0, *d1, *d2, *d3, *d4;
  int end[5];
};
__device__ __forceinline__ void copy_lds5(const LdsCopy5& c) {
  const int tot = c.end[4], bd = blockDim.x;
  for (int w0 = threadIdx.x; w0 < tot; w0 += 8 * bd) {
    int v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int w = min(w0 + q * bd, tot - 1);
      const int* sp = w < c.end[0] ? c.s0 + w
                    : w < c.end[1] ? c.s1 + (w - c.end[0])
                    : w < c.end[2] ? c.s2 + (w - c.end[1])
                    : w < c.end[3] ? c.s3 + (w - c.end[2])
                                   : c.s4 + (w - c.end[3]);
      v[q] = *sp;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int w = w0 + q * bd;
      if (w >= tot) continue;
      int* dp = w < c.end[0] ? c.d0 + w
              : w < c.end[1] ? c.d1 + (w - c.end[0])
              : w < c.end[2] ? c.d2 + (w - c.end[1])
              : w < c.end[3] ? c.d3 + (w - c.end[2])
                             : c.d4 + (w - c.end[3]);
      *dp = v[q];
    }
  }
}

// a segment is processed by a whole wavefront: keep its fields in scalar registers
__device__ __forceinline__ int ufl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ NDSeg uniform_seg(NDSeg a) {
  NDSeg b;
  b.m_off = ((long long)ufl((int)(a.m_off >> 32)) << 32) | (unsigned)ufl((int)(a.m_off & 0xffffffffLL));
  b.ld = ufl(a.ld);
  b.r0 = ufl(a.r0);
  b.nr = ufl(a.nr);
  b.k0 = ufl(a.k0);
  b.k1 = ufl(a.k1);
  b.vslot = ufl(a.vslot);
  b.pslot = ufl(a.pslot);
  b.pad = 0;
  return b;
}

// A segment of at most 16 (32) rows spreads 4 (2) groups of 16 columns over the wavefront:
// lane l takes row l mod g and columns k0 + 16 (l / g) .. + 16, g = lanes per group.
__device__ __forceinline__ int seg_group(const NDSeg& sg) { return sg.nr <= 16 ? 16 : sg.nr <= 32 ? 32 : 64; }

// the 16 matrix entries of a segment for one lane (row and column indices clamped)
template <typename C>
__device__ __forceinline__ void load_seg(const C* __restrict__ M, const NDSeg& sg, int lane, C* m) {
  const int gs = seg_group(sg), kq = sg.k0 + (lane / gs) * 16;
  const C* col = M + sg.m_off + sg.r0 + min(lane & (gs - 1), sg.nr - 1);
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) m[kk] = col[(long long)min(kq + kk, sg.k1 - 1) * sg.ld];
}

// Tree-block substitution: one work-group per subtree task, one stage per level.
//   gathers:  vec[slot] = src[rid] (+ children's updates)           all threads
//   segments: partial products of <= 64 rows over <= 16 columns       one wavefront, two at a time
//             (<= 32 rows over <= 32 columns, <= 16 rows over <= 64 columns)
//   outputs:  sum of a row block's partials, write x or the update    one wavefront each
// forward (FWD = 1): M = L = [A^-1; C A^-1] (ld ldL), src = r;  rows < nS give x_S = g_S,
//                    rows >= nS the update v_B - C A^-1 f_S of the parent
// backward:          M = W = -A^-1 B (ld ldW), src = x (the boundary solution);  x_S += W x_B
// The task's schedule is copied to LDS first, so a stage costs two dependent global
// accesses (gathered values, matrix entries) besides its barriers.
template <typename C, int FWD>
__global__ void __launch_bounds__(1024) k_nd_tree(const NDTask* __restrict__ tasks,
                                                  const NDStage* __restrict__ stages,
                                                  const NDGather* __restrict__ gath, const NDSeg* __restrict__ segs,
                                                  const NDOut* __restrict__ outs, const int* __restrict__ dst,
                                                  const int* __restrict__ cidx, const C* __restrict__ M,
                                                  C* __restrict__ upd, const C* __restrict__ src,
                                                  C* __restrict__ x, int conj, NDRhs rh) {
  typedef decltype(src[0].x) R;
  extern __shared__ __align__(16) char smem[];
  upd += blockIdx.y * rh.upd;          // right-hand side blockIdx.y
  src += blockIdx.y * rh.vec;
  x += blockIdx.y * rh.vec;
  const NDTask T = tasks[blockIdx.x];
  const int nst = T.st1 - T.st0, ng = T.g1 - T.g0, nsg = T.s1 - T.s0, no = T.o1 - T.o0, nd = T.d1 - T.d0;
  char* p = smem;
  NDStage* lst = (NDStage*)p;
  p += al16(sizeof(NDStage) * nst);
  NDGather* lg = (NDGather*)p;
  p += al16(sizeof(NDGather) * ng);
  NDSeg* lsg = (NDSeg*)p;
  p += al16(sizeof(NDSeg) * nsg);
  NDOut* lo = (NDOut*)p;
  p += al16(sizeof(NDOut) * no);
  int* ldst = (int*)p;
  p += al16(sizeof(int) * nd);
  // values forwarded between the task's levels: forward, the update vectors of fronts whose
  // parent is in the task; backward, the solution x_S of fronts with a descendant in it
  C* lupd = (C*)p;
  p += al16(sizeof(C) * T.nlu);
  C* lsrc = (C*)p;                     // per gather: r (forward) or x from outside the task
  p += al16(sizeof(C) * ng);
  C* lxg = (C*)p;                      // backward: x_S before the update, per output row
  p += al16(sizeof(C) * (FWD ? 0 : nd));
  C* work = (C*)p;
  // the launch-invariant inputs of the first 2 x blockDim gathers (and backward outputs)
  // take their indices from the schedule in global memory, so their loads overlap the copy
  const int bd = blockDim.x, tid = threadIdx.x;
  C pre[2], prx[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    pre[j] = prx[j] = mk((R)0, (R)0);
    if (ng > 0) {
      const NDGather g = gath[T.g0 + min(tid + j * bd, ng - 1)];
      const C v = src[max(g.rid, 0)];
      pre[j] = g.rid >= 0 && (FWD || g.u0 == -1) ? v : mk((R)0, (R)0);
    }
    if (!FWD && nd > 0) prx[j] = x[max(dst[T.d0 + min(tid + j * bd, nd - 1)], 0)];
  }
  {
    LdsCopy5 c;
    c.s0 = (const int*)(stages + T.st0);
    c.s1 = (const int*)(gath + T.g0);
    c.s2 = (const int*)(segs + T.s0);
    c.s3 = (const int*)(outs + T.o0);
    c.s4 = dst + T.d0;
    c.d0 = (int*)lst;
    c.d1 = (int*)lg;
    c.d2 = (int*)lsg;
    c.d3 = (int*)lo;
    c.d4 = ldst;
    c.end[0] = (int)(sizeof(NDStage) / 4) * nst;
    c.end[1] = c.end[0] + (int)(sizeof(NDGather) / 4) * ng;
    c.end[2] = c.end[1] + (int)(sizeof(NDSeg) / 4) * nsg;
    c.end[3] = c.end[2] + (int)(sizeof(NDOut) / 4) * no;
    c.end[4] = c.end[3] + nd;
    copy_lds5(c);
  }
  __syncthreads();
  const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // prefetching holds a second segment in registers: FP32 only (FP64 would spill).  The
  // first stage's segments are requested together with the launch-invariant inputs below.
  constexpr bool PF = sizeof(C) == 8;
  NDSeg psg;
  C pm[PF ? 16 : 1];
  bool have_pf = false;
  if (PF && nst > 0 && lst[0].s0 + wv < lst[0].s1) {
    psg = uniform_seg(lsg[lst[0].s0 + wv]);
    load_seg(M, psg, lane, pm);
    have_pf = true;
  }
  // every stage's inputs that do not change during the launch: r (forward); x of fronts
  // above the task and x_S before the update (backward)
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (tid + j * bd < ng) lsrc[tid + j * bd] = pre[j];
    if (!FWD && tid + j * bd < nd) lxg[tid + j * bd] = prx[j];
  }
  for (int e = tid + 2 * bd; e < ng; e += bd) {
    const NDGather g = lg[e];
    const C v = src[max(g.rid, 0)];
    lsrc[e] = g.rid >= 0 && (FWD || g.u0 == -1) ? v : mk((R)0, (R)0);
  }
  if (!FWD)
    for (int e = tid + 2 * bd; e < nd; e += bd) lxg[e] = x[max(ldst[e], 0)];
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const NDStage S = lst[st];
    // loads are unconditional (clamped indices, zero weights) so that a wavefront keeps
    // all of them in flight instead of waiting on each one
    for (int e = S.g0 + (int)threadIdx.x; e < S.g1; e += blockDim.x) {
      const NDGather g = lg[e];
      C v = mk((R)0, (R)0);
      if (FWD) {
        // rhs from LDS; contributions of the task's own fronts from LDS, of fronts below
        // the task (the previous launch) from global memory
        v = lsrc[e];
        if (g.u0 >= 0 || g.u1 >= 0) {
          const C u0 = upd[max(g.u0, 0)], u1 = upd[max(g.u1, 0)];
          if (g.u0 >= 0) v += u0;
          if (g.u1 >= 0) v += u1;
        }
        if (g.u0 <= -2) v += lupd[-g.u0 - 2];
        if (g.u1 <= -2) v += lupd[-g.u1 - 2];
        for (int q = g.ca; q < g.cb; ++q) v += upd[cidx[q]];
      } else {
        v = g.u0 <= -2 ? lupd[-g.u0 - 2] : lsrc[e];    // x_B: from a task level above, or prefetched
      }
      work[g.slot] = v;
    }
    __syncthreads();
    // one segment per wavefront at a time, 16 matrix loads in flight; the first segment of
    // a wavefront in a stage was prefetched during the previous stage (the matrix does not
    // depend on the previous stage's results)
    for (int s0 = S.s0 + wv; s0 < S.s1; s0 += nw) {
      NDSeg sg;
      C mv[16];
      if (PF && s0 == S.s0 + wv && have_pf) {
        sg = psg;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) mv[kk] = pm[PF ? kk : 0];
      } else {
        sg = uniform_seg(lsg[s0]);
        load_seg(M, sg, lane, mv);
      }
      const int gs = seg_group(sg), kq = sg.k0 + (lane / gs) * 16;
      C acc = mk((R)0, (R)0);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk)
        if (kq + kk < sg.k1) acc += cmul_conj(mv[kk], work[sg.vslot + kq + kk], conj);
      for (int o = gs; o < 64; o <<= 1) {      // sum the column groups (every lane gets its row's sum)
        acc.x += __shfl_xor(acc.x, o, 64);
        acc.y += __shfl_xor(acc.y, o, 64);
      }
      work[sg.pslot + lane] = acc;
    }
    // prefetch this wavefront's first segment of the next stage
    have_pf = false;
    if (PF && st + 1 < nst) {
      const NDStage S2 = lst[st + 1];
      if (S2.s0 + wv < S2.s1) {
        psg = uniform_seg(lsg[S2.s0 + wv]);
        load_seg(M, psg, lane, pm);
        have_pf = true;
      }
    }
    __syncthreads();
    for (int o = S.o0 + wv; o < S.o1; o += nw) {
      const NDOut ob = lo[o];
      if (lane < ob.nr) {
        C acc = mk((R)0, (R)0);
        for (int q = 0; q < ob.nparts; ++q) acc += work[ob.pslot + 64 * q + lane];
        const int d = ldst[ob.d + lane];
        if (FWD) {
          if (d >= 0) {
            x[d] = acc;
          } else {
            const C u = work[ob.vslot + ob.r0 + lane] - acc;
            upd[-d - 1] = u;
            if (ob.lu_on) lupd[ob.lu + lane] = u;   // row >= nS: read by the parent's gather
          }
        } else {
          const C nx = lxg[ob.d + lane] + acc;
          x[d] = nx;
          if (ob.lu_on) lupd[ob.lu + lane] = nx;     // read by the gathers of lower levels
        }
      }
    }
    __syncthreads();
  }
}

// rows [r0, r1) (at most 16) of a big front: 16 row lanes x KS (16 or 64) k-splits per
// work-group, partial sums reduced through LDS; consecutive threads read consecutive rows
// of one column.  gemv16_load issues the thread's first 16 matrix entries, which do not
// depend on v, so callers start it before gathering v; gemv16_finish does the rest.
template <typename C, int KS = 16>
__device__ __forceinline__ void gemv16_load(const C* __restrict__ M, long long ld, int r0, int r1, int K, C* m) {
  const int row = threadIdx.x & 15, ks = threadIdx.x >> 4;
  const int kq = (K + KS - 1) / KS, kb = ks * kq, ke = min(K, kb + kq);
  const C* col = M + min(r0 + row, r1 - 1);
#pragma unroll
  for (int q = 0; q < 16; ++q) m[q] = col[(long long)max(0, min(kb + q, ke - 1)) * ld];
}
template <typename C, int KS = 16>
__device__ __forceinline__ C gemv16_finish(const C* __restrict__ M, long long ld, int r0, int r1, int K,
                                           const C* __restrict__ v, int conj, C* red, const C* m0) {
  typedef decltype(v[0].x) R;
  const int row = threadIdx.x & 15, ks = threadIdx.x >> 4;
  const int i = r0 + row;
  const int kq = (K + KS - 1) / KS, kb = ks * kq, ke = min(K, kb + kq);
  C acc = mk((R)0, (R)0);
  if (i < r1 && kb < ke) {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (kb + q < ke) acc += cmul_conj(m0[q], v[kb + q], conj);
    // 16 matrix entries in flight per thread: load all (clamped), then accumulate
    const C* col = M + i;
    for (int k = kb + 16; k < ke; k += 16) {
      C m[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) m[q] = col[(long long)min(k + q, ke - 1) * ld];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (k + q < ke) acc += cmul_conj(m[q], v[k + q], conj);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (KS > 16) {                       // fold the k-splits 16 apart onto the first 256 threads
    C t = mk((R)0, (R)0);
    if (threadIdx.x < 256) {
      t = red[threadIdx.x];
#pragma unroll
      for (int g = 1; g < KS / 16; ++g) t += red[threadIdx.x + 256 * g];
    }
    __syncthreads();
    if (threadIdx.x < 256) red[threadIdx.x] = t;
    __syncthreads();
  }
  C tot = mk((R)0, (R)0);
  if (threadIdx.x < 16)
    for (int q = 0; q < 16; ++q) tot += red[q * 16 + threadIdx.x];
  return tot;
}

// forward substitution, big fronts: one work-group per chunk of at most 16 rows; KS = 64
// (1024 threads) as for the backward substitution
template <typename C, int KS>
__global__ void __launch_bounds__(16 * KS) k_nd_fwd_big(const NDGather* __restrict__ gath, const int* __restrict__ idx,
                                                         const int* __restrict__ cidx, const C* __restrict__ Lp,
                                                         C* __restrict__ upd, const NDItem* __restrict__ items,
                                                         const C* __restrict__ r, C* __restrict__ x,
                                                         C* __restrict__ gvec, int cap, int conj, NDRhs rh) {
  extern __shared__ char smem[];
  __shared__ C red[16 * KS];
  upd += blockIdx.y * rh.upd;
  r += blockIdx.y * rh.vec;
  x += blockIdx.y * rh.vec;
  C* vec = gvec ? gvec + blockIdx.y * rh.gvec + (long long)blockIdx.x * cap : (C*)smem;
  const NDItem f = items[blockIdx.x];
  const int* id = idx + f.idx_off;
  C m0[16];
  gemv16_load<C, KS>(Lp + f.m_off, f.ld, f.r0, f.r1, f.nS, m0);
  const NDGather* gl = gath + f.g0;
  for (int i = threadIdx.x; i < f.nS; i += 16 * KS) vec[i] = gather_list(gl[i], cidx, upd, r);
  for (int i = max(f.r0, f.nS) + threadIdx.x; i < f.r1; i += 16 * KS) vec[i] = gather_list(gl[i], cidx, upd, r);
  __syncthreads();
  C acc = gemv16_finish<C, KS>(Lp + f.m_off, f.ld, f.r0, f.r1, f.nS, vec, conj, red, m0);
  const int i = f.r0 + threadIdx.x;
  if (threadIdx.x < 16 && i < f.r1) {
    if (i < f.nS)
      x[id[i]] = acc;
    else
      upd[f.upd_off + i - f.nS] = vec[i] - acc;
  }
}

// backward substitution, big fronts: one work-group per chunk of at most 16 rows; KS = 64
// (1024 threads) for launches whose vectors exceed 256 entries and whose work-groups fit
// the chip at once (see big_threads), so that the gather of x_B takes one pass and a
// thread's k-slice one batch of loads
template <typename C, int KS>
__global__ void __launch_bounds__(16 * KS) k_nd_bwd_big(const NDFrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                         const C* __restrict__ Wp, const NDItem* __restrict__ items,
                                                         C* __restrict__ x, C* __restrict__ gvec, int cap, int conj,
                                                         NDRhs rh) {
  extern __shared__ char smem[];
  __shared__ C red[16 * KS];
  x += blockIdx.y * rh.vec;
  C* vec = gvec ? gvec + blockIdx.y * rh.gvec + (long long)blockIdx.x * cap : (C*)smem;
  const NDItem f = items[blockIdx.x];
  const int* id = idx + f.idx_off;
  C m0[16];
  gemv16_load<C, KS>(Wp + f.m_off, f.ld, f.r0, f.r1, f.nB, m0);
  const int i = f.r0 + threadIdx.x;
  const int di = threadIdx.x < 16 && i < f.r1 ? id[i] : 0;
  for (int j = threadIdx.x; j < f.nB; j += 16 * KS) vec[j] = x[id[f.nS + j]];
  __syncthreads();
  C acc = gemv16_finish<C, KS>(Wp + f.m_off, f.ld, f.r0, f.r1, f.nB, vec, conj, red, m0);
  if (threadIdx.x < 16 && i < f.r1) x[di] = x[di] + acc;
}

// ---- split-K launches (kind 3) -------------------------------------------
// P[pslot + t] = sum_{k0 <= k < k1} M[k ld + r0 + t] vec[k]: one row per thread, 16 loads in
// flight.  The tile gathers its own k-slice of the front's input vector from the gather list
// (entry voff + k is the front's entry k), so no separate gather launch and buffer pass is
// needed; tiles of the same k-slice repeat its 128 gathers, which are small beside the
// 256 x 128 matrix block each of them streams.
template <typename C, int FWD>
__global__ void __launch_bounds__(256) k_nd_tile(const NDFrontDev* __restrict__ fr, const C* __restrict__ Mp,
                                                 const NDTile* __restrict__ tiles, const NDGather* __restrict__ gath,
                                                 const int* __restrict__ cidx, const C* __restrict__ upd,
                                                 const C* __restrict__ src, C* __restrict__ P, int conj, NDRhs rh) {
  typedef decltype(src[0].x) R;
  __shared__ C vec[128];
  upd += blockIdx.y * rh.upd;
  src += blockIdx.y * rh.vec;
  P += blockIdx.y * rh.part;
  const NDTile t = tiles[blockIdx.x];
  const NDFrontDev f = fr[t.front];
  const int ld = FWD ? f.ldL : f.ldW, rows = FWD ? f.nF : f.nS;
  const int nk = t.k1 - t.k0;
  const int i = min(t.r0 + (int)threadIdx.x, rows - 1);
  const C* col = Mp + (FWD ? f.L_off : f.W_off) + (long long)t.k0 * ld + i;
  // the first 16 matrix entries do not depend on the gathered slice: request them first
  C m0[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) m0[q] = col[(long long)min(q, nk - 1) * ld];
  if ((int)threadIdx.x < nk) vec[threadIdx.x] = gather_list(gath[t.voff + t.k0 + threadIdx.x], cidx, upd, src);
  __syncthreads();
  C acc = mk((R)0, (R)0);
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q < nk) acc += cmul_conj(m0[q], vec[q], conj);
  for (int k = 16; k < nk; k += 16) {
    C m[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) m[q] = col[(long long)min(k + q, nk - 1) * ld];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (k + q < nk) acc += cmul_conj(m[q], vec[k + q], conj);
  }
  P[t.pslot + threadIdx.x] = acc;
}

// rows of a row tile: the partials summed in k order, then x (or the update) written; the
// forward update rows gather their own input entry
template <typename C, int FWD>
__global__ void __launch_bounds__(256) k_nd_rowsum(const NDFrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                   const NDRowTile* __restrict__ rt, const C* __restrict__ P,
                                                   const NDGather* __restrict__ gath, const int* __restrict__ cidx,
                                                   const C* __restrict__ src, C* __restrict__ upd,
                                                   C* __restrict__ x, NDRhs rh) {
  typedef decltype(src[0].x) R;
  P += blockIdx.y * rh.part;
  upd += blockIdx.y * rh.upd;
  src += blockIdx.y * rh.vec;
  x += blockIdx.y * rh.vec;
  const NDRowTile t = rt[blockIdx.x];
  const NDFrontDev f = fr[t.front];
  const int i = t.r0 + threadIdx.x;
  if (i >= (FWD ? f.nF : f.nS)) return;
  C acc = mk((R)0, (R)0);
  // in k order; groups of 8 loads are issued before their sums, so they are in flight together
  const C* pp = P + t.pslot + threadIdx.x;
  int q = 0;
  for (; q + 8 <= t.nkt; q += 8) {
    C v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pp[256 * (q + u)];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; q < t.nkt; ++q) acc += pp[256 * q];
  if (FWD) {
    if (i < f.nS)
      x[idx[f.idx_off + i]] = acc;
    else
      upd[f.upd_off + i - f.nS] = gather_list(gath[t.voff + i], cidx, (const C*)upd, src) - acc;
  } else {
    const int id = idx[f.idx_off + i];
    x[id] = x[id] + acc;
  }
}

template <typename C, int FWD>
static void splitk(const NDLaunchDev& L, const NDFrontDev* fr, const int* idx, const int* cidx, const C* M, C* upd,
                   const C* src, C* x, C* P, int conj, const NDRhs& rh, hipStream_t s) {
  hipLaunchKernelGGL((k_nd_tile<C, FWD>), dim3(L.ntiles, rh.n), dim3(256), 0, s, fr, M, L.tiles, L.gath, cidx,
                     (const C*)upd, src, P, conj, rh);
  hipLaunchKernelGGL((k_nd_rowsum<C, FWD>), dim3(L.nrt, rh.n), dim3(256), 0, s, fr, idx, L.rtiles, (const C*)P,
                     L.gath, cidx, src, upd, x, rh);
}

// ------------------------------------------------------------- launchers ----
void nd_zero(cd* p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_d2, dim3(2048), dim3(256), 0, s, p, n);
}
void nd_iota(int* perm, const NDFrontDev* fr, int nfronts, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(nfronts), dim3(64), 0, s, perm, fr, nfronts);
}
void nd_assemble(const NDFrontDev* fr, const int* ids, int nids, int max_asm, const NDAsm* asmv,
                 const cd* coef, cd* Fp, hipStream_t s) {
  unsigned gx = (unsigned)std::min(1024, std::max(1, (max_asm + 255) / 256));
  hipLaunchKernelGGL(k_nd_assemble, dim3(gx, nids), dim3(256), 0, s, fr, ids, asmv, coef, Fp);
}
void nd_extend(const NDFrontDev* fr, const int* ids, int nids, long long max_nb2, const int* children,
               const long long* child_map_off, const int* maps, cd* Fp, int slot, hipStream_t s) {
  unsigned gx = (unsigned)std::min<long long>(2048, std::max<long long>(1, (max_nb2 + 255) / 256));
  hipLaunchKernelGGL(k_nd_extend, dim3(gx, nids), dim3(256), 0, s, fr, ids, children, child_map_off, maps, Fp, slot);
}
void nd_panel_multi(const NDFrontDev* fr, int nids, int max_nF, cd* Fp, cd* Pb, int* perm, int* swp,
                    PivCand* cand, int k0, int kb, int max_nS, int* err, hipStream_t s) {
  const int nblk = (max_nF + PROWS - 1) / PROWS;
  const int kbb = std::min(kb, max_nS - k0);
  const long long pstride = (long long)nblk * PROWS * kb;     // panel-buffer entries per front
  PivCand* cbuf[2] = {cand, cand + (size_t)nids * nblk};
  hipLaunchKernelGGL(k_piv_search, dim3(nblk, nids), dim3(256), 0, s, fr, nullptr, Fp, k0, cbuf[0], nblk);
  for (int kk = 0; kk < kbb; ++kk) {
    if (kb > 32)
      hipLaunchKernelGGL(k_piv_step<64>, dim3(nblk, nids), dim3(256), 0, s, fr, Fp, Pb, pstride, kk & 1, k0, kb, kk,
                         cbuf[kk & 1], cbuf[(kk + 1) & 1], nblk, perm, swp, err);
    else
      hipLaunchKernelGGL(k_piv_step<32>, dim3(nblk, nids), dim3(256), 0, s, fr, Fp, Pb, pstride, kk & 1, k0, kb, kk,
                         cbuf[kk & 1], cbuf[(kk + 1) & 1], nblk, perm, swp, err);
  }
  hipLaunchKernelGGL(k_piv_back, dim3(nblk, nids), dim3(256), 0, s, fr, Fp, Pb, pstride, k0, kb);
  unsigned gx = (unsigned)std::min(64, std::max(1, (max_nF + 255) / 256));
  hipLaunchKernelGGL(k_nd_swap_rest, dim3(gx, nids), dim3(256), 0, s, fr, nullptr, Fp, swp, k0, kb);
}
void nd_panel_reg(const NDFrontDev* fr, const int* ids, int nids, int max_nF, cd* Fp, int* perm, int* swp, int k0,
                  int kb, int* err, hipStream_t s) {
  // variants: rows per thread R x panel width KB <= 32 entries in registers
  if (kb == 32 && max_nF <= 128)
    hipLaunchKernelGGL((k_nd_panel_reg<32, 1, 128>), dim3(nids), dim3(128), 0, s, fr, ids, Fp, perm, swp, k0, err);
  else if (kb == 32 && max_nF <= 256)
    hipLaunchKernelGGL((k_nd_panel_reg<32, 1, 256>), dim3(nids), dim3(256), 0, s, fr, ids, Fp, perm, swp, k0, err);
  else if (kb == 16 && max_nF <= 512)
    hipLaunchKernelGGL((k_nd_panel_reg<16, 2, 256>), dim3(nids), dim3(256), 0, s, fr, ids, Fp, perm, swp, k0, err);
  else if (kb == 16 && max_nF <= 1024)
    hipLaunchKernelGGL((k_nd_panel_reg<16, 2, 512>), dim3(nids), dim3(512), 0, s, fr, ids, Fp, perm, swp, k0, err);
  else if (kb == 8 && max_nF <= 2048)
    hipLaunchKernelGGL((k_nd_panel_reg<8, 4, 512>), dim3(nids), dim3(512), 0, s, fr, ids, Fp, perm, swp, k0, err);
  else
    throw std::runtime_error("register panel: unsupported front size / panel width");
  unsigned gx = (unsigned)std::min(64, std::max(1, (max_nF + 255) / 256));
  hipLaunchKernelGGL(k_nd_swap_rest, dim3(gx, nids), dim3(256), 0, s, fr, ids, Fp, swp, k0, kb);
}
void nd_save_t(const NDFrontDev* fr, const int* ids, int nids, const long long* toff, long long max_n,
               cd* Fp, cd* T, int k0, int kb, int u0, int un, hipStream_t s) {
  unsigned gx = (unsigned)std::min<long long>(1024, std::max<long long>(1, (max_n + 255) / 256));
  hipLaunchKernelGGL(k_nd_save_t, dim3(gx, nids), dim3(256), 0, s, fr, ids, toff, Fp, T, k0, kb, u0, un);
}
void nd_gemm(const NDFrontDev* fr, const int* ids, int nids, const long long* toff, int max_rows, int max_cols,
             cd* Fp, const cd* T, int k0, int kb, int u0, int un, hipStream_t s) {
  int tiles = ((max_rows + GT - 1) / GT) * ((max_cols + GT - 1) / GT);
  hipLaunchKernelGGL(k_nd_gemm, dim3(tiles, nids), dim3(256), 0, s, fr, ids, toff, Fp, T, k0, kb, u0, un);
}
template <typename C>
void nd_finalize(const NDFrontDev* fr, const int* ids, int nids, long long max_n, const cd* Fp,
                 const int* perm, C* Lp, C* Wp, hipStream_t s) {
  unsigned gx = (unsigned)std::min<long long>(1024, std::max<long long>(1, (max_n + 255) / 256));
  hipLaunchKernelGGL((k_nd_finalize<C>), dim3(gx, nids), dim3(256), 0, s, fr, ids, Fp, perm, Lp, Wp);
}
// LDS bytes above the default limit need the attribute on the kernel
template <typename C, int FWD>
static void tree_attr(size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_nd_tree<C, FWD>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// threads of a row-chunk launch: 1024 (64 k-splits) where the plan marks its vectors as
// longer than 256 entries and at most 512 work-groups run (two 16-wavefront work-groups
// per CU: one generation); otherwise 256.  A second generation doubles the launch's
// latency, which cost more than the shorter gather and k-slices save.
static int big_threads(const NDLaunchDev& L, const NDRhs& rh) {
  return L.threads == 1024 && (long long)L.ntasks * rh.n <= 512 ? 1024 : 256;
}

template <typename C>
void nd_fwd(const NDLaunchDev& L, const NDFrontDev* fr, const int* idx, const int* cptr, const int* cidx,
            const C* Lp, C* upd, const C* r, C* x, C* gvec, int cap, int conj, C* P, const NDRhs& rh,
            hipStream_t s) {
  if (L.kind == 3) {
    splitk<C, 1>(L, fr, idx, cidx, Lp, upd, r, x, P, conj, rh, s);
  } else if (L.kind == 2) {
    size_t lds = (size_t)L.lds_bytes;
    tree_attr<C, 1>(lds);
    hipLaunchKernelGGL((k_nd_tree<C, 1>), dim3(L.ntasks, rh.n), dim3(L.threads), lds, s, L.tasks, L.stages, L.gath,
                       L.segs, L.outs, L.dst, cidx, Lp, upd, r, x, conj, rh);
  } else {
    if (big_threads(L, rh) == 1024)
      hipLaunchKernelGGL((k_nd_fwd_big<C, 64>), dim3(L.ntasks, rh.n), dim3(1024), L.shm, s, L.gath, idx, cidx, Lp,
                         upd, L.items, r, x, gvec, cap, conj, rh);
    else
      hipLaunchKernelGGL((k_nd_fwd_big<C, 16>), dim3(L.ntasks, rh.n), dim3(256), L.shm, s, L.gath, idx, cidx, Lp,
                         upd, L.items, r, x, gvec, cap, conj, rh);
  }
}
template <typename C>
void nd_bwd(const NDLaunchDev& L, const NDFrontDev* fr, const int* idx, const int* cidx, const C* Wp, C* upd, C* x,
            C* gvec, int cap, int conj, C* P, const NDRhs& rh, hipStream_t s) {
  if (L.kind == 3) {
    splitk<C, 0>(L, fr, idx, cidx, Wp, upd, (const C*)x, x, P, conj, rh, s);
  } else if (L.kind == 2) {
    size_t lds = (size_t)L.lds_bytes;
    tree_attr<C, 0>(lds);
    hipLaunchKernelGGL((k_nd_tree<C, 0>), dim3(L.ntasks, rh.n), dim3(L.threads), lds, s, L.tasks, L.stages, L.gath,
                       L.segs, L.outs, L.dst, cidx, Wp, upd, (const C*)x, x, conj, rh);
  } else {
    if (big_threads(L, rh) == 1024)
      hipLaunchKernelGGL((k_nd_bwd_big<C, 64>), dim3(L.ntasks, rh.n), dim3(1024), L.shm, s, fr, idx, Wp, L.items, x,
                         gvec, cap, conj, rh);
    else
      hipLaunchKernelGGL((k_nd_bwd_big<C, 16>), dim3(L.ntasks, rh.n), dim3(256), L.shm, s, fr, idx, Wp, L.items, x,
                         gvec, cap, conj, rh);
  }
}

template void nd_finalize<cf>(const NDFrontDev*, const int*, int, long long, const cd*, const int*,
                                  cf*, cf*, hipStream_t);
template void nd_finalize<cd>(const NDFrontDev*, const int*, int, long long, const cd*, const int*,
                                   cd*, cd*, hipStream_t);
template void nd_fwd<cf>(const NDLaunchDev&, const NDFrontDev*, const int*, const int*, const int*, const cf*, cf*,
                         const cf*, cf*, cf*, int, int, cf*, const NDRhs&, hipStream_t);
template void nd_fwd<cd>(const NDLaunchDev&, const NDFrontDev*, const int*, const int*, const int*, const cd*, cd*,
                         const cd*, cd*, cd*, int, int, cd*, const NDRhs&, hipStream_t);
template void nd_bwd<cf>(const NDLaunchDev&, const NDFrontDev*, const int*, const int*, const cf*, cf*, cf*, cf*, int,
                         int, cf*, const NDRhs&, hipStream_t);
template void nd_bwd<cd>(const NDLaunchDev&, const NDFrontDev*, const int*, const int*, const cd*, cd*, cd*, cd*, int,
                         int, cd*, const NDRhs&, hipStream_t);


}  // namespace helm
