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

__global__ void __launch_bounds__(256) k_nd_extend(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                   const int* __restrict__ maps, cd* __restrict__ Fp, int slot) {
  const NDFrontDev f = fr[ids[blockIdx.y]];
  int c = f.child[slot];
  if (c < 0) return;
  const NDFrontDev fc = fr[c];
  long long n2 = (long long)fc.nB * fc.nB;
  const int* mp = maps + f.map_off[slot];
  cd* F = Fp + f.F_off;
  const cd* Fc = Fp + fc.F_off;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n2; p += (long long)gridDim.x * blockDim.x) {
    int k1 = (int)(p / fc.nB), k2 = (int)(p % fc.nB);
    F[(long long)mp[k1] * f.nF + mp[k2]] += Fc[(long long)(fc.nS + k1) * fc.nF + fc.nS + k2];
  }
}

// panel [k0, k0 + kbb) of every front of one height: one work-group per front
__global__ void __launch_bounds__(256) k_nd_panel(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                  cd* __restrict__ Fp, int* __restrict__ perm, int k0, int kb,
                                                  int* __restrict__ err) {
  const NDFrontDev f = fr[ids[blockIdx.x]];
  if (f.nS <= k0) return;
  const int kbb = min(kb, f.nS - k0);
  const int nF = f.nF;
  cd* F = Fp + f.F_off;
  int* pm = perm + f.perm_off;
  __shared__ double s_val[256];
  __shared__ int s_idx[256];
  __shared__ cd s_rk[64];
  const int tid = threadIdx.x;
  for (int k = k0; k < k0 + kbb; ++k) {
    // pivot: largest |F[i][k]| among the not yet exchanged S rows i >= k
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < f.nS; i += blockDim.x) {
      double v = abs2(F[(long long)i * nF + k]);
      if (v > best) { best = v; bi = i; }
    }
    s_val[tid] = best;
    s_idx[tid] = bi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (tid < w) {
        double o = s_val[tid + w];
        int oi = s_idx[tid + w];
        if (o > s_val[tid] || (o == s_val[tid] && oi < s_idx[tid])) { s_val[tid] = o; s_idx[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = s_idx[0];
    const double pv = s_val[0];
    __syncthreads();
    if (p != k) {
      for (int j = tid; j < nF; j += blockDim.x) {
        cd t = F[(long long)k * nF + j];
        F[(long long)k * nF + j] = F[(long long)p * nF + j];
        F[(long long)p * nF + j] = t;
      }
      if (tid == 0) {
        int t = pm[k];
        pm[k] = pm[p];
        pm[p] = t;
      }
      __syncthreads();
    }
    if (tid < kbb) s_rk[tid] = F[(long long)k * nF + k0 + tid];
    __syncthreads();
    cd piv = s_rk[k - k0];
    if (!(pv > 0.0)) {
      if (tid == 0) atomicOr(err, 1);
      piv = mk(1.0, 0.0);
    }
    const cd inv = cdiv(mk(1.0, 0.0), piv);
    for (int i = tid; i < nF; i += blockDim.x) {
      if (i == k) continue;
      cd* row = F + (long long)i * nF + k0;
      cd ck = row[k - k0] * inv;      // F'[i][k] = F[i][k] / piv
      for (int jj = 0; jj < kbb; ++jj) {
        if (jj == k - k0) continue;
        row[jj] -= ck * s_rk[jj];
      }
      row[k - k0] = ck;
    }
    if (tid < kbb) {
      cd* rowk = F + (long long)k * nF + k0;
      if (tid == k - k0)
        rowk[tid] = inv;
      else
        rowk[tid] = -(s_rk[tid] * inv);
    }
    __syncthreads();
  }
}

// T = F[K rows][J columns] (J = all columns outside K), then zero those entries
__global__ void __launch_bounds__(256) k_nd_save_t(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                   const long long* __restrict__ toff, cd* __restrict__ Fp,
                                                   cd* __restrict__ T, int k0, int kb) {
  const NDFrontDev f = fr[ids[blockIdx.y]];
  if (f.nS <= k0) return;
  const int kbb = min(kb, f.nS - k0);
  const int ncol = f.nF - kbb;
  cd* F = Fp + f.F_off;
  cd* Tt = T + toff[blockIdx.y];
  long long n = (long long)kbb * ncol;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
    int kk = (int)(p / ncol), jj = (int)(p % ncol);
    int j = jj < k0 ? jj : jj + kbb;
    long long a = (long long)(k0 + kk) * f.nF + j;
    Tt[p] = F[a];
    F[a] = mk(0.0, 0.0);
  }
}

// F[:, J] -= F[:, K] * T   (complex FP64 GEMM, 64x64 tiles, 4x4 per thread)
#define GT 64
#define GK 16
__global__ void __launch_bounds__(256) k_nd_gemm(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                 const long long* __restrict__ toff, cd* __restrict__ Fp,
                                                 const cd* __restrict__ T, int k0, int kb) {
  const NDFrontDev f = fr[ids[blockIdx.y]];
  if (f.nS <= k0) return;
  const int kbb = min(kb, f.nS - k0);
  const int M = f.nF, Ncol = f.nF - kbb;
  const int tilesN = (Ncol + GT - 1) / GT, tilesM = (M + GT - 1) / GT;
  if ((int)blockIdx.x >= tilesM * tilesN) return;
  const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;
  cd* F = Fp + f.F_off;
  const cd* Tt = T + toff[blockIdx.y];
  __shared__ cd sA[GK][GT + 1];
  __shared__ cd sB[GK][GT + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  cd acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = mk(0.0, 0.0);
  for (int kk0 = 0; kk0 < kbb; kk0 += GK) {
    for (int p = threadIdx.x; p < GK * GT; p += 256) {
      int kk = p % GK, r = p / GK;                 // A tile: consecutive threads along a row
      int row = tm * GT + r, kq = kk0 + kk;
      sA[kk][r] = (row < M && kq < kbb) ? F[(long long)row * f.nF + k0 + kq] : mk(0.0, 0.0);
      int kk2 = p / GT, c = p % GT;                // B tile: consecutive threads along a row of T
      int col = tn * GT + c, kq2 = kk0 + kk2;
      sB[kk2][c] = (col < Ncol && kq2 < kbb) ? Tt[(long long)kq2 * Ncol + col] : mk(0.0, 0.0);
    }
    __syncthreads();
    for (int kk = 0; kk < GK; ++kk) {
      cd a[4], b[4];
      for (int q = 0; q < 4; ++q) {
        a[q] = sA[kk][ty + 16 * q];
        b[q] = sB[kk][tx + 16 * q];
      }
      for (int qa = 0; qa < 4; ++qa)
        for (int qb = 0; qb < 4; ++qb) acc[qa][qb] += a[qa] * b[qb];
    }
    __syncthreads();
  }
  for (int qa = 0; qa < 4; ++qa) {
    int row = tm * GT + ty + 16 * qa;
    if (row >= M) continue;
    for (int qb = 0; qb < 4; ++qb) {
      int col = tn * GT + tx + 16 * qb;
      if (col >= Ncol) continue;
      int j = col < k0 ? col : col + kbb;
      F[(long long)row * f.nF + j] -= acc[qa][qb];
    }
  }
}

template <typename C>
__global__ void __launch_bounds__(256) k_nd_finalize(const NDFrontDev* __restrict__ fr, const int* __restrict__ ids,
                                                     const cd* __restrict__ Fp, const int* __restrict__ perm,
                                                     C* __restrict__ Lp, C* __restrict__ Wp) {
  const NDFrontDev f = fr[ids[blockIdx.y]];
  const cd* F = Fp + f.F_off;
  const int* pm = perm + f.perm_off;
  long long nL = (long long)f.nF * f.nS, nW = (long long)f.nS * f.nB;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nL + nW;
       p += (long long)gridDim.x * blockDim.x) {
    if (p < nL) {
      int i = (int)(p / f.nS), k = (int)(p % f.nS);
      Lp[f.L_off + (long long)i * f.nS + pm[k]] = conv<C>::from(F[(long long)i * f.nF + k]);
    } else {
      long long q = p - nL;
      int i = (int)(q / f.nB), j = (int)(q % f.nB);
      Wp[f.W_off + q] = conv<C>::from(F[(long long)i * f.nF + f.nS + j]);
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
__device__ __forceinline__ C cfma_conj(C a, C x, int conj) {   // (conj? conj(a) : a) * x
  if (conj) a.y = -a.y;
  return a * x;
}

template <typename C>
__device__ __forceinline__ C wave_sum(C v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

template <typename C>
__global__ void __launch_bounds__(256) k_nd_fwd(const NDFrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                const int* __restrict__ maps, const C* __restrict__ Lp,
                                                C* __restrict__ upd, const int* __restrict__ task_off,
                                                const NDItem* __restrict__ items, const C* __restrict__ r,
                                                C* __restrict__ x, C* __restrict__ gvec, int vec_cap, int conj) {
  extern __shared__ char smem[];
  C* vec = gvec ? gvec + (long long)blockIdx.x * vec_cap : (C*)smem;
  typedef decltype(vec[0].x) R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int it = task_off[blockIdx.x]; it < task_off[blockIdx.x + 1]; ++it) {
    const NDItem item = items[it];
    const NDFrontDev f = fr[item.front];
    const int* id = idx + f.idx_off;
    for (int i = tid; i < f.nF; i += 256) {
      vec[i] = i < f.nS ? r[id[i]] : mk((R)0, (R)0);
    }
    __syncthreads();
    for (int s = 0; s < 2; ++s) {
      int c = f.child[s];
      if (c < 0) continue;
      const NDFrontDev fc = fr[c];
      const int* mp = maps + f.map_off[s];
      const C* u = upd + fc.upd_off;
      for (int k = tid; k < fc.nB; k += 256) vec[mp[k]] += u[k];
      __syncthreads();
    }
    const C* L = Lp + f.L_off;
    for (int i = item.r0 + wv; i < item.r1; i += 4) {
      const C* row = L + (long long)i * f.nS;
      C acc = mk((R)0, (R)0);
      for (int k = lane; k < f.nS; k += 64) acc += cfma_conj(row[k], vec[k], conj);
      acc = wave_sum(acc);
      if (lane == 0) {
        if (i < f.nS)
          x[id[i]] = acc;
        else
          upd[f.upd_off + i - f.nS] = vec[i] - acc;
      }
    }
    __syncthreads();
  }
}

template <typename C>
__global__ void __launch_bounds__(256) k_nd_bwd(const NDFrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                const C* __restrict__ Wp, const int* __restrict__ task_off,
                                                const NDItem* __restrict__ items, C* __restrict__ x,
                                                C* __restrict__ gvec, int vec_cap, int conj) {
  extern __shared__ char smem[];
  C* vec = gvec ? gvec + (long long)blockIdx.x * vec_cap : (C*)smem;
  typedef decltype(vec[0].x) R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int it = task_off[blockIdx.x]; it < task_off[blockIdx.x + 1]; ++it) {
    const NDItem item = items[it];
    const NDFrontDev f = fr[item.front];
    const int* id = idx + f.idx_off;
    for (int j = tid; j < f.nB; j += 256) vec[j] = x[id[f.nS + j]];
    __syncthreads();
    const C* W = Wp + f.W_off;
    for (int i = item.r0 + wv; i < item.r1; i += 4) {
      const C* row = W + (long long)i * f.nB;
      C acc = mk((R)0, (R)0);
      for (int k = lane; k < f.nB; k += 64) acc += cfma_conj(row[k], vec[k], conj);
      acc = wave_sum(acc);
      if (lane == 0) x[id[i]] = x[id[i]] + acc;
    }
    __syncthreads();
  }
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
void nd_extend(const NDFrontDev* fr, const int* ids, int nids, long long max_nb2, const int* maps, cd* Fp,
               int slot, hipStream_t s) {
  unsigned gx = (unsigned)std::min<long long>(2048, std::max<long long>(1, (max_nb2 + 255) / 256));
  hipLaunchKernelGGL(k_nd_extend, dim3(gx, nids), dim3(256), 0, s, fr, ids, maps, Fp, slot);
}
void nd_panel(const NDFrontDev* fr, const int* ids, int nids, cd* Fp, int* perm, int k0, int kb, int* err,
              hipStream_t s) {
  hipLaunchKernelGGL(k_nd_panel, dim3(nids), dim3(256), 0, s, fr, ids, Fp, perm, k0, kb, err);
}
void nd_save_t(const NDFrontDev* fr, const int* ids, int nids, const long long* toff, long long max_n,
               cd* Fp, cd* T, int k0, int kb, hipStream_t s) {
  unsigned gx = (unsigned)std::min<long long>(1024, std::max<long long>(1, (max_n + 255) / 256));
  hipLaunchKernelGGL(k_nd_save_t, dim3(gx, nids), dim3(256), 0, s, fr, ids, toff, Fp, T, k0, kb);
}
void nd_gemm(const NDFrontDev* fr, const int* ids, int nids, const long long* toff, int max_nF, cd* Fp,
             const cd* T, int k0, int kb, hipStream_t s) {
  int tiles = ((max_nF + GT - 1) / GT) * ((max_nF + GT - 1) / GT);
  hipLaunchKernelGGL(k_nd_gemm, dim3(tiles, nids), dim3(256), 0, s, fr, ids, toff, Fp, T, k0, kb);
}
template <typename C>
void nd_finalize(const NDFrontDev* fr, const int* ids, int nids, long long max_n, const cd* Fp,
                 const int* perm, C* Lp, C* Wp, hipStream_t s) {
  unsigned gx = (unsigned)std::min<long long>(1024, std::max<long long>(1, (max_n + 255) / 256));
  hipLaunchKernelGGL((k_nd_finalize<C>), dim3(gx, nids), dim3(256), 0, s, fr, ids, Fp, perm, Lp, Wp);
}
template <typename C>
void nd_fwd(int ntasks, size_t lds, const NDFrontDev* fr, const int* idx, const int* maps, const C* Lp, C* upd,
            const int* task_off, const NDItem* items, const C* r, C* x, C* gvec, int vec_cap, int conj,
            hipStream_t s) {
  hipLaunchKernelGGL((k_nd_fwd<C>), dim3(ntasks), dim3(256), lds, s, fr, idx, maps, Lp, upd, task_off, items, r, x,
                     gvec, vec_cap, conj);
}
template <typename C>
void nd_bwd(int ntasks, size_t lds, const NDFrontDev* fr, const int* idx, const C* Wp, const int* task_off,
            const NDItem* items, C* x, C* gvec, int vec_cap, int conj, hipStream_t s) {
  hipLaunchKernelGGL((k_nd_bwd<C>), dim3(ntasks), dim3(256), lds, s, fr, idx, Wp, task_off, items, x, gvec, vec_cap,
                     conj);
}

template void nd_finalize<cf>(const NDFrontDev*, const int*, int, long long, const cd*, const int*,
                                  cf*, cf*, hipStream_t);
template void nd_finalize<cd>(const NDFrontDev*, const int*, int, long long, const cd*, const int*,
                                   cd*, cd*, hipStream_t);
template void nd_fwd<cf>(int, size_t, const NDFrontDev*, const int*, const int*, const cf*, cf*,
                             const int*, const NDItem*, const cf*, cf*, cf*, int, int, hipStream_t);
template void nd_fwd<cd>(int, size_t, const NDFrontDev*, const int*, const int*, const cd*, cd*,
                              const int*, const NDItem*, const cd*, cd*, cd*, int, int, hipStream_t);
template void nd_bwd<cf>(int, size_t, const NDFrontDev*, const int*, const cf*, const int*, const NDItem*,
                             cf*, cf*, int, int, hipStream_t);
template void nd_bwd<cd>(int, size_t, const NDFrontDev*, const int*, const cd*, const int*,
                              const NDItem*, cd*, cd*, int, int, hipStream_t);

}  // namespace helm
