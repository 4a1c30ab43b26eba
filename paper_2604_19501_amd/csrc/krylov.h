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
  int its, done, nonfinite, pad;
  double hist[KMAXIT];
  cd G[(KMAXM + 1) * (KMAXM + 1)];   // Gram matrix of the stored basis, leading dimension KMAXM + 1
};

struct KrylovArgs {
  FineOp op;
  cd s;           // omega^2 (the unshifted outer operator)
  int conj;
  const double* m64;
  cd* V;          // basis, restart + 1 vectors
  long long ldv;
  cd* part;       // partial sums, value-major: part[i * pcap + block]
  int pcap;
  int nblk;            // blocks of the node kernels = ceil(N / (256 * KNPT))
  KrylovState* st;
};

void kr_init(const KrylovArgs& a, hipStream_t s);
void kr_residual(const KrylovArgs& a, const cd* x, const cd* b, int with_b, hipStream_t s);
void kr_scale_v0(const KrylovArgs& a, hipStream_t s);
void kr_arnoldi(const KrylovArgs& a, const void* z, int z_f32, int j, double tol, hipStream_t s);
void kr_update_x(const KrylovArgs& a, const void* Z, int z_f32, long long ldz, int k, cd* x, hipStream_t s);
void kr_zero(cd* x, long long n, hipStream_t s);

}  // namespace helm
