// Device state and launch arguments of the FGMRES kernels (internal).
#pragma once
#include "internal.h"

namespace helm {

#define KMAXM 64
#define KMAXIT 4096
#define KNPT 4            // nodes per thread in the reduction kernels

struct KrylovState {
  cd H[(KMAXM + 1) * KMAXM];   // Hessenberg, column-major, leading dimension KMAXM + 1
  double cs[KMAXM];
  cd sn[KMAXM];
  cd g[KMAXM + 1];
  cd y[KMAXM];
  cd h1[2 * KMAXM + 3];          // sums of the dot pass: h1, Gram column, ||w||^2
  cd c[KMAXM + 1];               // Hessenberg column before rotation (h1 + h2)
  cd tmp[2];
  double bnorm, beta0, est, hnext, true_rel;
  int its, done;
  int final;          // set by the host when this right-hand side is finished: every later
                      // restart keeps it done
  int nonfinite;
  int kcols;          // Arnoldi columns completed in the current cycle
  int maxit;          // iteration limit (the column that reaches it ends the solve)
  double hist[KMAXIT];
  cd G[(KMAXM + 1) * (KMAXM + 1)];   // Gram matrix of the stored basis, leading dimension KMAXM + 1
  int ticket;         // blocks of the current final-sum launch that have stored their sum
};

// nrhs right-hand sides are iterated in lock-step (grid y): right-hand side r has state
// st[r], basis vector j at V + j ldv + r N (ldv = nrhs N) and its partial sums at
// part + r pstride; the other vectors of right-hand side r follow those of r - 1 at N.
struct KrylovArgs {
  FineOp op;
  cd s;           // omega^2 (the unshifted outer operator)
  int conj;
  const double* m64;
  cd* V;          // basis, restart + 1 vectors per right-hand side
  long long ldv;
  cd* part;       // partial sums, value-major: part[i * pcap + block]
  int pcap;
  int nblk;            // blocks of the node kernels = ceil(N / (256 * KNPT))
  KrylovState* st;
  int nrhs;
  long long pstride;
  double guard;        // ||w - V c||^2 below guard ||w||^2 ends the restart cycle (cancellation)
};

void kr_init(const KrylovArgs& a, int max_iter, hipStream_t s);
void kr_residual(const KrylovArgs& a, const cd* x, const cd* b, int with_b, hipStream_t s);
void kr_scale_v0(const KrylovArgs& a, hipStream_t s);
// pack_dst: host-mapped slot that receives the scalar blocks of the states after the
// column's Givens update (as kr_pack_states; written by the update pass); null: none.
// fused: the final sums and the Givens update in one launch (the last block of each
// right-hand side's sums finishing the column behind device-scope fences); else two
void kr_arnoldi(const KrylovArgs& a, const void* z, int z_f32, int j, double tol, void* pack_dst, int fused,
                hipStream_t s);
// x += Z y over each right-hand side's columns of the current cycle (Z: ldz between columns)
void kr_update_x(const KrylovArgs& a, const void* Z, int z_f32, long long ldz, cd* x, hipStream_t s);
// x += z (the stationary iteration's update; z in cycle precision)
void kr_add_z(const KrylovArgs& a, const void* z, int z_f32, cd* x, hipStream_t s);
void kr_zero(cd* x, long long n, hipStream_t s);
// timing runs: hold the stream for about rounds x 3.4 us
void kr_hold(int rounds, hipStream_t s);
// copy the nrhs scalar blocks (bnorm .. hist) into host memory mapped for the device
void kr_pack_states(const KrylovArgs& a, void* host_dst, hipStream_t s);
// mark the right-hand sides of a bit mask finished (their kernels do nothing from now on)
void kr_finalize(const KrylovArgs& a, unsigned mask, hipStream_t s);

}  // namespace helm
