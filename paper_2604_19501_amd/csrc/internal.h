// Internal declarations of libhelm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>

#include "../../include/helm.h"

namespace helm {

// ---------------------------------------------------------------------------
// complex numbers: interleaved (re, im) in FP32 (cf) and FP64 (cd).  Dedicated
// types rather than HIP's float2/double2, whose operators are element-wise.
// ---------------------------------------------------------------------------
struct __align__(8) cf { float x, y; };
struct __align__(16) cd { double x, y; };
template <typename R> struct cplx;
template <> struct cplx<float> { typedef cf type; };
template <> struct cplx<double> { typedef cd type; };

__host__ __device__ inline cf mk(float a, float b) { cf r; r.x = a; r.y = b; return r; }
__host__ __device__ inline cd mk(double a, double b) { cd r; r.x = a; r.y = b; return r; }
__host__ __device__ inline cf operator+(cf a, cf b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cd operator+(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cf operator-(cf a, cf b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cd operator-(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cf operator-(cf a) { return mk(-a.x, -a.y); }
__host__ __device__ inline cd operator-(cd a) { return mk(-a.x, -a.y); }
__host__ __device__ inline cf operator*(cf a, cf b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cd operator*(cd a, cd b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cf operator*(float s, cf a) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline cd operator*(double s, cd a) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline cf& operator+=(cf& a, cf b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cd& operator+=(cd& a, cd b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cf& operator-=(cf& a, cf b) { a.x -= b.x; a.y -= b.y; return a; }
__host__ __device__ inline cd& operator-=(cd& a, cd b) { a.x -= b.x; a.y -= b.y; return a; }
__host__ __device__ inline cf conjc(cf a) { return mk(a.x, -a.y); }
__host__ __device__ inline cd conjc(cd a) { return mk(a.x, -a.y); }
__host__ __device__ inline float abs2(cf a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double abs2(cd a) { return a.x * a.x + a.y * a.y; }
// a * conj(b) and conj(a) * b
__host__ __device__ inline cd cmulc(cd a, cd b) {  // conj(a) * b
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cf cmulc(cf a, cf b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cd cdiv(cd a, cd b) {
  double d = b.x * b.x + b.y * b.y;
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__host__ __device__ inline cf cdiv(cf a, cf b) {
  float d = b.x * b.x + b.y * b.y;
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
// conversions between precisions
__host__ __device__ inline cf to_f(cd a) { return mk((float)a.x, (float)a.y); }
__host__ __device__ inline cf to_f(cf a) { return a; }
__host__ __device__ inline cd to_d(cf a) { return mk((double)a.x, (double)a.y); }
__host__ __device__ inline cd to_d(cd a) { return a; }
// streaming accesses of vectors that a pass reads or writes once (the Krylov basis):
// marked non-temporal so that they do not displace the data reused from pass to pass
// (the coarsest factors, the level-2 coefficients) in the caches
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cd ld_nt(const cd* p) {
  const dvec2 v = __builtin_nontemporal_load((const dvec2*)p);
  return mk(v.x, v.y);
}
__device__ __forceinline__ void st_nt(cd* p, cd v) {
  dvec2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, (dvec2*)p);
}

template <typename C> struct conv;
template <> struct conv<cf> {
  __host__ __device__ static cf from(cd a) { return to_f(a); }
  __host__ __device__ static cf from(cf a) { return a; }
};
template <> struct conv<cd> {
  __host__ __device__ static cd from(cd a) { return a; }
  __host__ __device__ static cd from(cf a) { return to_d(a); }
};

// ---------------------------------------------------------------------------
// grid geometry of one level
// ---------------------------------------------------------------------------
struct Geom {
  int dim;
  int n[3];       // cells (1 node on unused axes: n = 0)
  int N[3];       // nodes per axis = n + 1 (1 on unused axes)
  long long tot;  // total nodes
};

// coordinates of flat node index f = i0 + N0 (i1 + N1 i2); a grid has fewer than 2^31 nodes,
// so 32-bit division serves (64-bit division has no instruction and costs some 40)
__device__ __forceinline__ void node_coords(const Geom& g, long long f, int& i0, int& i1, int& i2) {
  const unsigned u = (unsigned)f, N0 = (unsigned)g.N[0], N1 = (unsigned)g.N[1];
  const unsigned r = u / N0;
  i0 = (int)(u - r * N0);
  const unsigned q = r / N1;
  i1 = (int)(r - q * N1);
  i2 = (int)q;
}

inline Geom make_geom(int dim, const int* n) {
  Geom g;
  g.dim = dim;
  g.tot = 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = a < dim ? n[a] : 0;
    g.N[a] = g.n[a] + 1;
    g.tot *= g.N[a];
  }
  return g;
}
inline Geom coarsen(const Geom& f) {
  int n[3] = {f.n[0] / 2, f.n[1] / 2, f.n[2] / 2};
  return make_geom(f.dim, n);
}

// fine level operator: -Lap_h - s * m (1 - i sigma) with a complex scalar s
struct FineOp {
  Geom g;
  int compact = 0;      // 1: the compact fourth-order operator (eqs. 3.1, 3.2) with its mass term
  double inv_h2;
  int layer[3][2];
  double sigma_max;
  // the layer profile's per-axis constants (set by set_layer_profile): reciprocal widths
  // (0 where a face has no layer) in FP64 and FP32, and the first node past the high face's
  // inner edge
  double inv_w[3][2];
  float inv_wf[3][2];
  int inner_hi[3];
};

// the profile's constants of op.layer and op.g
inline void set_layer_profile(FineOp& op) {
  for (int a = 0; a < 3; ++a) {
    for (int s = 0; s < 2; ++s) {
      const int w = a < op.g.dim ? op.layer[a][s] : 0;
      op.inv_w[a][s] = w > 0 ? 1.0 / w : 0.0;
      op.inv_wf[a][s] = (float)op.inv_w[a][s];
    }
    op.inner_hi[a] = op.g.n[a] - (a < op.g.dim ? op.layer[a][1] : 0);
  }
}

// sigma = sigma_max * sum over axes of (depth into the layer / width)^2, without branches:
// the depth below the low face's inner edge is max(lo - i, 0), past the high face's
// max(i - (n - hi), 0), and a face without a layer has reciprocal width 0
__host__ __device__ inline double layer_sigma(const FineOp& op, int i0, int i1, int i2) {
  const int ii[3] = {i0, i1, i2};
  double s = 0.0;
  for (int a = 0; a < op.g.dim; ++a) {
    const double tl = (double)max(op.layer[a][0] - ii[a], 0) * op.inv_w[a][0];
    const double th = (double)max(ii[a] - op.inner_hi[a], 0) * op.inv_w[a][1];
    s += tl * tl + th * th;
  }
  return op.sigma_max * s;
}

// number of stencil points of the stored coarse operators
__host__ __device__ inline int stencil_points(int dim) { return dim == 2 ? 9 : 27; }

// ---------------------------------------------------------------------------
// nested-dissection structure of the coarsest level (host side)
// ---------------------------------------------------------------------------
struct NDFrontDev {
  int nS, nB, nF;
  int nchild;           // children: plan.children[child_off .. child_off + nchild)
  int child_off;
  int height;
  long long idx_off;    // nF ints: S nodes then B nodes (level-3 flat indices)
  long long inv_off;    // nF+1 ints at cptr[inv_off]: contributions to position i are
                        // cidx[cptr[i] .. cptr[i+1]) (absolute indices into the update pool)
  long long F_off;      // nF*nF cd (row major), setup scratch; holds Schur block for parent
  long long L_off;      // nF x nS column major (ld ldL): left block column [A^-1; C A^-1] (cycle precision)
  long long W_off;      // nS x nB column major (ld ldW): top-right block -A^-1 B          (cycle precision)
  long long upd_off;    // nB update vector (cycle precision)
  long long perm_off;   // nS ints
  long long asm_off;    // assembly entries
  int asm_cnt;
  // leading dimensions of L and W: nF and nS rounded up to 128 bytes, with L_off and W_off
  // multiples of 128 bytes, so that a column run of a row chunk starts on a cache line
  int ldL, ldW;
  int pad;
};

#define ND_KBMAX 64     // widest factorisation panel (columns)
#define ND_KBOUT 128    // widest column block of the trailing exchange update

struct PivCand {        // a row block's pivot candidate: largest |F[i][k]| and its row
  double v;
  int i, pad;
};

struct NDAsm {          // F[row][col] += coef[cidx]
  int row, col;
  long long cidx;
};

struct NDItem {         // one work item of a multi-block launch: rows [r0, r1) of a front
  int front, r0, r1;
  int stage;
  // the front's fields the work item needs (copied, so a work-group reads one record)
  int nS, nF, nB;
  int g0;               // forward: the front's gather list (one entry per front row) in the launch's gath
  int ld, pad;          // leading dimension of the block (ldL forward, ldW backward)
  long long m_off;      // L_off (forward) or W_off (backward)
  long long idx_off, inv_off, upd_off;
};

// Tree-block launches: one work-group walks the fronts of a subtree level by level.
// Per level ("stage"): gather the fronts' input vectors into LDS, partial matrix-vector
// products over row blocks of at most 64 rows and k ranges of at most 16 ("segments",
// one wavefront each), then sum the partials of every row block and write the results
// ("outputs").  A work-group first copies its task's schedule into LDS; indices inside
// a task are relative to the task's first gather / segment / output / destination.
struct NDTask {
  int st0, st1, g0, g1, s0, s1, o0, o1, d0, d1;
  int nlu;              // forward: entries of the LDS copy of the task's internal update vectors
  int pad;
};
struct NDStage {
  int g0, g1, s0, s1, o0, o1;
};
struct NDGather {       // vec[slot] = (rid >= 0 ? src[rid] : 0) + upd[u0] + upd[u1] + sum upd[cidx[ca .. cb))
  int slot, rid, u0, u1, ca, cb;   // u0, u1: -1 none; <= -2 (tree blocks): LDS update entry -u - 2
};
struct NDSeg {          // part[pslot + l] = sum_{k0 <= k < k1} M[m_off + k ld + r0 + l] vec[vslot + k], l < nr
  long long m_off;
  int ld, r0, nr, k0, k1, vslot, pslot, pad;
};
struct NDOut {          // rows [r0, r0 + nr): y = sum of nparts partial blocks of 64; destinations dst[d ..)
  int r0, nr, vslot, pslot, nparts, d;   // dst >= 0: x index; dst < 0: update index -dst - 1
  int lu, lu_on;        // lu_on: row r0 + l's update also goes to LDS update entry lu + l
};

// Split-K launches for heights with large fronts: every front's input vector is gathered
// once (flat gather list -> gather buffer), tiles of 256 rows x at most 128 columns write
// partial products (one row per thread, so a column is read in 2 KB runs), and row
// tiles sum their partials in a fixed order and write x or the update.
struct NDTile {
  int front, r0, k0, k1;
  int pslot;            // partial sums P[pslot + t], t < 256
  int voff;             // the front's first entry in the flat gather list
};
struct NDRowTile {
  int front, r0, nkt, pslot, voff, pad;
};

struct NDLaunch {       // one kernel launch of a substitution
  int kind = 1;         // 1: row chunks of big fronts (one work-group per item); 2: tree blocks;
                        // 3: split-K tiles (gather, tiles, row sums: three kernels)
  std::vector<int> task_off;   // kind 1: items[task_off[t] ..); kind 2: stages[task_off[t] ..)
  std::vector<NDItem> items;
  int max_rows_vec = 0; // kind 1: vector entries per work-group (nF forward, nB backward)
  std::vector<NDTask> tasks;
  std::vector<NDStage> stages;
  std::vector<NDGather> gath;
  std::vector<NDSeg> segs;
  std::vector<NDOut> outs;
  std::vector<int> dst;
  std::vector<NDTile> tiles;        // kind 3 (with gath: the flat gather list)
  std::vector<NDRowTile> rtiles;
  long long p_elems = 0;
  int lds_bytes = 0;    // kind 2: schedule + vectors + partials per work-group
  int threads = 256;
};

// several right-hand sides substituted by one launch (grid y): strides, in entries,
// between the vectors of consecutive right-hand sides
struct NDRhs {
  int n = 1;             // right-hand sides
  int pad = 0;
  long long vec = 0;     // r and x (N3)
  long long upd = 0;     // update pool
  long long part = 0;    // split-K partial products
  long long gvec = 0;    // row-chunk launches' global vectors
};

struct NDLaunchDev {    // device copy of an NDLaunch, as the kernels see it
  int kind = 1, ntasks = 0, threads = 256, lds_bytes = 0;
  size_t shm = 0;       // kind 1: dynamic LDS bytes for the gathered vector (0: global fall-back)
  const int* task_off = nullptr;
  const NDItem* items = nullptr;
  const NDTask* tasks = nullptr;
  const NDStage* stages = nullptr;
  const NDGather* gath = nullptr;
  const NDSeg* segs = nullptr;
  const NDOut* outs = nullptr;
  const int* dst = nullptr;
  int ngath = 0, ntiles = 0, nrt = 0;
  const NDTile* tiles = nullptr;
  const NDRowTile* rtiles = nullptr;
};

struct NDPlan {
  Geom g;                               // level-3 geometry
  std::vector<NDFrontDev> fronts;
  std::vector<int> idx, maps, cptr, cidx, children;
  std::vector<long long> child_map_off;   // per entry of `children`: offset of its map
  int max_children = 0;
  std::vector<NDAsm> asmv;
  std::vector<std::vector<int>> by_height;   // front ids per height
  int max_height = 0;
  long long F_total = 0, L_total = 0, W_total = 0, upd_total = 0, perm_total = 0;
  long long L_alloc = 0, W_alloc = 0;   // entries of the padded L and W storage
  long long T_scratch = 0;              // doubles2 of panel row buffer (max over heights)
  int max_nS = 0, max_nB = 0, max_nF = 0;
  std::vector<NDLaunch> fwd, bwd;
  std::vector<int> cuts;                // heights closing the tree-block launches
};

// elem_bytes: bytes of a factor entry (cycle precision); lds_bytes: LDS available to a
// tree block; cuts: heights closing the tree-block launches (empty: chosen by the cost
// model, {-1}: no tree blocks)
// splitk_bytes: heights above the tree blocks whose factor blocks hold at least this many
// bytes (per direction) use split-K launches
// tree_waves: the most wavefronts of a tree-block work-group (16 = 1024 threads)
// merge_heights: heights of the dissection tree (leaves 0, before any merge) whose fronts are
// merged into their parents (fewer levels, larger fronts)
// radius: stencil radius of the coarsest operator (its (2 radius + 1)^dim coefficient planes,
// plane k of offset d = sum_a (d_a + radius) (2 radius + 1)^a)
void nd_plan(const Geom& g3, int leaf_max, int rows_chunk, int root_merge, int elem_bytes, int lds_bytes,
             const std::vector<int>& cuts, long long splitk_bytes, NDPlan& plan, int tree_waves = 16,
             const std::vector<int>& merge_heights = std::vector<int>(), int radius = 1);


}  // namespace helm
