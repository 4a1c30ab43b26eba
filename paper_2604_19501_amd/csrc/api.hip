// C ABI of libhelm: validation, workspace layout, setup, cycle and FGMRES drivers.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdarg>
#include <cstdlib>
#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "krylov.h"
#include "levels_api.h"
#include "wide.h"

namespace helm {

// launchers implemented in the kernel files
void gal_fine(const FineOp& op, cd s, const double* m, const Geom& gc, cd* out, hipStream_t st);
void gal_coarse(const Geom& g, const cd* A, const Geom& gc, cd* out, hipStream_t st);
void cast_d2f(const cd* a, cf* b, long long n, hipStream_t st);
void cast_f2d(const cf* a, cd* b, long long n, hipStream_t st);
void square_slowness(const double* kap, double* m64, float* m32, long long n, int is_m, hipStream_t st);
void nd_zero(cd* p, long long n, hipStream_t s);
void nd_iota(int* perm, const NDFrontDev* fr, int nfronts, hipStream_t s);
void nd_assemble(const NDFrontDev* fr, const int* ids, int nids, int max_asm, const NDAsm* asmv, const cd* coef,
                 cd* Fp, hipStream_t s);
void nd_extend(const NDFrontDev* fr, const int* ids, int nids, long long max_nb2, const int* children,
               const long long* child_map_off, const int* maps, cd* Fp, int slot, hipStream_t s);
// Fp: the fronts; Pb: a panel buffer of max_nF (rounded to 32) x kb entries per front;
// cand: two candidate sets of nids x ceil(max_nF / 32)
void nd_panel_multi(const NDFrontDev* fr, int nids, int max_nF, cd* Fp, cd* Pb, int* perm, int* swp,
                    PivCand* cand, int k0, int kb, int max_nS, int* err, hipStream_t s);
void nd_save_t(const NDFrontDev* fr, const int* ids, int nids, const long long* toff, long long max_n, cd* Fp,
               cd* T, int k0, int kb, int u0, int un, hipStream_t s);
void nd_gemm(const NDFrontDev* fr, const int* ids, int nids, const long long* toff, int max_rows, int max_cols,
             cd* Fp, const cd* T, int k0, int kb, int u0, int un, hipStream_t s);
template <typename C>
void nd_finalize(const NDFrontDev* fr, const int* ids, int nids, long long max_n, const cd* Fp, const int* perm,
                 C* Lp, C* Wp, hipStream_t s);
template <typename C>
void nd_fwd(const NDLaunchDev& L, const NDFrontDev* fr, const int* idx, const int* cptr, const int* cidx,
            const C* Lp, C* upd, const C* r, C* x, C* gvec, int cap, int conj, C* P, const NDRhs& rh, hipStream_t s);
int panel_reg_kb(int nF);
void nd_panel_reg(const NDFrontDev* fr, const int* ids, int nids, int max_nF, cd* Fp, int* perm, int* swp, int k0,
                  int kb, int* err, hipStream_t s);
template <typename C>
void nd_bwd(const NDLaunchDev& L, const NDFrontDev* fr, const int* idx, const int* cidx, const C* Wp, C* upd, C* x,
            C* gvec, int cap, int conj, C* P, const NDRhs& rh, hipStream_t s);
void grad_accumulate(const FineOp& op, double omega, const cd* u, const cd* lam, double* g, int first,
                     hipStream_t s);

}  // namespace helm

using namespace helm;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

struct DevErr : std::runtime_error {
  using std::runtime_error::runtime_error;
};
#define CK(x)                                                                                        \
  do {                                                                                               \
    hipError_t e_ = (x);                                                                             \
    if (e_ != hipSuccess) throw DevErr(std::string(#x) + ": " + hipGetErrorString(e_));              \
  } while (0)

const size_t ALIGN = 256;
inline size_t al(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// linear carve of the workspace (base = 0 computes the size)
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    size_t o = off;
    off = al(off + count * sizeof(T));
    return base ? (T*)(base + o) : nullptr;
  }
};

struct NDDev {        // device-side ND tables (pointers into the workspace)
  NDFrontDev* fronts = nullptr;
  NDFrontDev* hfr = nullptr;   // fronts in height order
  int *idx = nullptr, *maps = nullptr, *cptr = nullptr, *cidx = nullptr, *perm = nullptr, *hlist = nullptr,
      *err = nullptr, *swp = nullptr;
  int* children = nullptr;
  long long* child_map_off = nullptr;
  NDAsm* asmv = nullptr;
  long long* toff = nullptr;
  cd *F = nullptr, *T = nullptr, *pb = nullptr;   // pb: multi-work-group panel buffer
  PivCand* cand = nullptr;
  void *L = nullptr, *W = nullptr;
  std::vector<NDLaunchDev> launch[2];   // forward, backward
  int gvec_cap = 0;
  long long part_n = 1, gvec_n = 0;   // entries per right-hand side of part, gvec
};

// Per-call scratch of one cycle: the iterates and right-hand sides of levels 1-3 and the
// coarsest solve's update pool, global gather vectors (launches whose vectors do not fit
// in LDS) and split-K partial products.  Nothing in it needs to
// start at zero: every entry is written before it is read within the call.  Sized for
// rc right-hand sides in lock-step.
struct CycleScratch {
  void *x1a = nullptr, *x1b = nullptr, *b2 = nullptr, *x2a = nullptr, *x2b = nullptr, *b3 = nullptr,
       *x3 = nullptr;
  void *upd = nullptr, *gvec = nullptr, *part = nullptr;
};

// kernel classes timed with HIP events when timing is on
enum KClass { KT_L1_SWEEP, KT_L1_RESTRICT, KT_L2_SWEEP, KT_L2_RESTRICT, KT_ND_FWD, KT_ND_BWD, KT_APPLY_DOT,
              KT_UPDATE_DOT, KT_NORMALIZE, KT_KRYLOV_OTHER, KT_L2_CHAIN, KT_TAIL, KT_N };
struct Pending {
  int cls;
  hipEvent_t a, b;
  int launches;       // kernel launches between the two events
};

struct HeightInfo {
  int start, count, max_asm, max_nS, max_nF, max_child;
  long long max_nb2, max_T, max_fin;
  long long f_bytes;      // the fronts' dense matrices, FP64 complex
};

}  // namespace

struct helm_ctx {
  helm_grid grid;
  helm_shift shift;
  helm_mg mg;
  double omega;
  Geom g1, g2, g3;
  FineOp op;
  int f32;              // cycle precision is FP32
  size_t csz;           // bytes of one complex in cycle precision
  // the coarsest solve's factors, vectors and substitution kernels in FP64 (nd64) or in the
  // cycle's precision, and their bytes per complex
  int nd64 = 0;
  size_t ndsz = 16;
  // device state
  double *m64 = nullptr;
  float* m32 = nullptr;
  cf* dg32 = nullptr;   // FP32 cycle: diagonal of the level-1 operator H_beta
  cd *coef2_64 = nullptr, *coef3_64 = nullptr, *tmp2 = nullptr;
  cf* coef2_32 = nullptr;
  CycleScratch scr;     // the cycle's scratch in the workspace
  cd *r3d = nullptr, *e3d = nullptr;
  NDPlan plan;
  NDDev nd;
  std::vector<HeightInfo> hinfo;
  std::vector<long long> hlist_toff;
  std::vector<int> hlist;
  // Krylov
  cd *V = nullptr, *part = nullptr;
  void* Z = nullptr;
  KrylovState* st = nullptr;
  // right-hand sides solved in lock-step: capacity (buffers are carved for it) and the
  // count of the current solve; with a capacity above 1, contiguous copies of the
  // right-hand sides and solutions
  int rcap = 1, nr = 1;
  int tail_fused = 1;   // the FGMRES tail as one launch (kr_arnoldi)
  int l2_chain = 1;     // 2D: level-2 post-sweep, next pre-sweep and restriction fused (HELM_L2_CHAIN)
  cd *Bm = nullptr, *Xm = nullptr;
  KrylovArgs ka;
  size_t ws_needed = 0;
  char* hstate = nullptr;    // pinned host copy of the scalar blocks of the states (slot 0),
                             // slots 1, 2: read-backs of alternate queued iterations
  char* hstate_dev = nullptr;   // its device mapping
  hipEvent_t itev[2] = {nullptr, nullptr};   // completion of the queued iterations
  int timing = 0;
  double times[5] = {0, 0, 0, 0, 0};
  double kt_ms[KT_N] = {0};
  long long kt_cnt[KT_N] = {0};
  std::vector<Pending> pending;
  std::vector<hipEvent_t> evpool;
  size_t lds_limit = 65536;     // LDS bytes for substitution vectors
  size_t lds_panel = 0;         // LDS bytes for a resident factorisation panel (device maximum - 2 KB)
  bool tuned = false;           // schedule parameters came from the autotuner cache
  int nd_leaf = 0, nd_root = 0;  // nested-dissection leaf size and root merge limit in use
  // the compact fourth-order stack: restriction (tr) and interpolating-restriction (ip, P =
  // 2^d ip^T) weights between levels 1-2 and 2-3, and the stencil radii and coefficient
  // planes of the stored level-2 and level-3 operators (radius 1 for the 5/7-point stack)
  int compact = 0;
  Transfer1D tr[2], ip[2];
  int r2 = 1, r3 = 1, K2 = 9, K3 = 9;
  long long nd_merge = 0;        // bit h: fronts of dissection height h merged into their parents
  // box-shape variants of the tiled cycle kernels: level-1 sweep, level-1 restriction,
  // level-2 sweep, level-2 restriction (levels.hip lists the shapes)
  int box[4] = {0, 0, 0, 0};
  std::vector<helm_ctx*> sub;   // batched form: one context per instance
  std::vector<hipStream_t> bstreams;   // batched form: streams of the concurrent instances
  // one captured graph per (operator, Arnoldi index j): cycle on V_j + Arnoldi step
  hipStream_t cap = nullptr;    // library-owned stream used only for capture
  std::vector<hipGraphExec_t> gexec[2];
  double gtol[2] = {-1.0, -1.0};
  int gnr[2] = {0, 0};          // right-hand side count the graphs were captured for
  int graphs = 1;
  double arnoldi_guard = 1e-8;  // relative size of ||w - V c||^2 below which an Arnoldi column ends the cycle
};

namespace {

int validate(const helm_grid* g, const helm_mg* mg) {
  if (!g || !mg) return fail(HELM_EINVAL, "grid or mg is NULL");
  if (g->dim != 2 && g->dim != 3) return fail(HELM_EINVAL, "dim must be 2 or 3 (got %d)", g->dim);
  for (int a = 0; a < g->dim; ++a) {
    if (g->n[a] < 4 || g->n[a] % 4 != 0) return fail(HELM_EINVAL, "n[%d] = %d must be a positive multiple of 4", a, g->n[a]);
    if (g->n[a] > (1 << 20)) return fail(HELM_EINVAL, "n[%d] too large", a);
    for (int s = 0; s < 2; ++s)
      if (g->layer[a][s] < 0) return fail(HELM_EINVAL, "negative layer width");
    if (g->layer[a][0] + g->layer[a][1] > g->n[a]) return fail(HELM_EINVAL, "layers wider than the grid on axis %d", a);
  }
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(HELM_EINVAL, "h must be positive and finite");
  if (!(g->sigma_max >= 0.0) || !std::isfinite(g->sigma_max)) return fail(HELM_EINVAL, "sigma_max must be >= 0");
  if (mg->cycle != 1 && mg->cycle != 2) return fail(HELM_EINVAL, "cycle must be 1 (V) or 2 (W)");
  if (mg->nu_pre < 0 || mg->nu_pre > 4 || mg->nu_post < 0 || mg->nu_post > 4)
    return fail(HELM_EINVAL, "nu_pre/nu_post must be in 0..4");
  for (int l = 0; l < 2; ++l)
    if (!std::isfinite(mg->jacobi[l])) return fail(HELM_EINVAL, "jacobi weight not finite");
  if (mg->cycle_prec != HELM_F64 && mg->cycle_prec != HELM_F32) return fail(HELM_EINVAL, "cycle_prec must be HELM_F64 or HELM_F32");
  if (mg->restart < 1 || mg->restart > KMAXM) return fail(HELM_EINVAL, "restart must be in 1..%d", KMAXM);
  if (mg->stack != HELM_STACK_P5 && mg->stack != HELM_STACK_COMPACT)
    return fail(HELM_EINVAL, "stack must be HELM_STACK_P5 or HELM_STACK_COMPACT");
  if (mg->stack == HELM_STACK_COMPACT) {
    if (mg->transfer != HELM_TRANSFER_CUBIC && mg->transfer != HELM_TRANSFER_LEVDEP)
      return fail(HELM_EINVAL, "the compact stack takes HELM_TRANSFER_CUBIC or HELM_TRANSFER_LEVDEP");
    if (g->dim == 3 && mg->transfer != HELM_TRANSFER_LEVDEP)
      return fail(HELM_EINVAL, "3D compact stack: level-dependent transfers only (cubic ones give a 343-point level-3 operator)");
  }
  long long N1 = 1;
  for (int a = 0; a < g->dim; ++a) N1 *= (g->n[a] + 1);
  if (N1 > (1LL << 31) - 1) return fail(HELM_EINVAL, "grid too large (N1 > 2^31-1)");
  return HELM_OK;
}

// kernels one substitution step launches (a split-K step: tiles, row sums)
int nd_step_kernels(int kind) { return kind == 3 ? 2 : 1; }
int nd_kernels(const std::vector<NDLaunchDev>& Ls) {
  int k = 0;
  for (const NDLaunchDev& L : Ls) k += nd_step_kernels(L.kind);
  return k;
}

// the calls that work on one hierarchy refuse the parent of a batched context: its
// instances live in its sub-contexts, and it holds no device state of its own
int need_single(const helm_ctx* c, const char* who) {
  if (!c->sub.empty()) return fail(HELM_EINVAL, "%s takes a single-instance context (this one is batched)", who);
  return HELM_OK;
}

// the compact operator is not complex symmetric, so conj(H) is not its adjoint: its
// contexts take HELM_OP_N only
int need_op(const helm_ctx* c, int op, const char* who) {
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (c->compact && op == HELM_OP_C)
    return fail(HELM_EINVAL, "%s: the compact stack has no adjoint path (HELM_OP_C)", who);
  return HELM_OK;
}

void init_geometry(helm_ctx* c) {
  int n[3] = {c->grid.n[0], c->grid.n[1], c->grid.dim == 3 ? c->grid.n[2] : 0};
  c->g1 = make_geom(c->grid.dim, n);
  c->g2 = coarsen(c->g1);
  c->g3 = coarsen(c->g2);
  c->op.g = c->g1;
  c->op.inv_h2 = 1.0 / (c->grid.h * c->grid.h);
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) c->op.layer[a][s] = a < c->grid.dim ? c->grid.layer[a][s] : 0;
  c->op.sigma_max = c->grid.sigma_max;
  set_layer_profile(c->op);
  c->f32 = c->mg.cycle_prec == HELM_F32;
  c->csz = c->f32 ? sizeof(cf) : sizeof(cd);
  c->compact = c->mg.stack == HELM_STACK_COMPACT;
  c->op.compact = c->compact;
  if (c->compact) {
    c->tr[0] = c->ip[0] = c->ip[1] = transfer_cubic();
    c->tr[1] = c->mg.transfer == HELM_TRANSFER_LEVDEP ? transfer_fw() : transfer_cubic();
    // Galerkin radii: a coarse row reaches (a_R + r_A + a_P) fine nodes, half as many coarse
    c->r2 = (c->tr[0].a + 1 + c->ip[0].a) / 2;
    c->r3 = (c->tr[1].a + c->r2 + c->ip[1].a) / 2;
  } else {
    c->r2 = c->r3 = 1;
  }
  // The compact stack's coarsest operator, shifted by its alpha* (1.0045 at G = 12), is close
  // to singular: at 1024^2 (257^2 coarsest nodes) its FP64 factors leave a relative residual
  // near 1e-8, so FP32 factors would give errors of order one.  Its coarsest solve keeps
  // FP64 factors with either cycle precision.
  c->nd64 = !c->f32 || c->compact;
  c->ndsz = c->nd64 ? sizeof(cd) : sizeof(cf);
  c->K2 = c->K3 = 1;
  for (int a = 0; a < c->grid.dim; ++a) {
    c->K2 *= 2 * c->r2 + 1;
    c->K3 *= 2 * c->r3 + 1;
  }
}

// planes of the FP32 level-2 coefficients: 3D keeps the symmetric half (centre onwards;
// the level kernels' Op2<3, float> reads them so)
static inline int sym2_planes(int dim) { return dim == 3 ? 14 : 9; }
const int ND_KB = ND_KBOUT;      // scratch of the exchange updates is sized for the widest column block
// nested-dissection parameters (tunable through the environment for the autotuner):
// leaf box size, rows per work-group of big fronts, nodes per subtree task
int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v && *v ? atoi(v) : dflt;
}

// schedule parameters of the coarsest solve picked by the autotuner: the JSON file named
// by HELM_TUNE_CACHE maps "nd:<dim>:<n0>x<n1>x<n2>:<f32|f64>" (the coarsest solve's
// precision; ":r<radius>" appended when the coarsest stencil radius is not 1) to an object
// with the integers "leaf", "root" and "splitk_kb" and the strings "cuts", "merge" and
// "boxes" among its members (others, nested objects and arrays included, are skipped);
// returns false when the file or the key is absent
struct TunedND {
  int leaf = -1, root = -1, splitk_kb = -1;
  std::string cuts, merge, boxes;
  bool has_cuts = false, has_merge = false, has_boxes = false;
};

// the members of the JSON object starting at txt[ob] == '{' that sit directly in it:
// name -> the raw text of the value (strings without their quotes)
std::map<std::string, std::string> json_members(const std::string& txt, size_t ob) {
  std::map<std::string, std::string> out;
  int depth = 0;
  size_t i = ob;
  std::string key;
  auto read_string = [&](size_t& p) {      // p at the opening quote; returns the content
    std::string v;
    for (++p; p < txt.size() && txt[p] != '"'; ++p) {
      if (txt[p] == '\\' && p + 1 < txt.size()) ++p;
      v += txt[p];
    }
    return v;                              // p at the closing quote
  };
  for (; i < txt.size(); ++i) {
    const char ch = txt[i];
    if (ch == '"') {
      std::string sv = read_string(i);
      if (depth == 1) {
        size_t k = i + 1;
        while (k < txt.size() && isspace((unsigned char)txt[k])) ++k;
        if (k < txt.size() && txt[k] == ':') {
          key = sv;                        // a member name; its value follows
          i = k;
          size_t v = k + 1;
          while (v < txt.size() && isspace((unsigned char)txt[v])) ++v;
          if (v < txt.size() && txt[v] == '"') {
            out[key] = read_string(v);
            i = v;
          } else if (v < txt.size() && txt[v] != '{' && txt[v] != '[') {
            size_t e = v;
            while (e < txt.size() && txt[e] != ',' && txt[e] != '}' && !isspace((unsigned char)txt[e])) ++e;
            out[key] = txt.substr(v, e - v);
            i = e - 1;
          }
        }
      }
    } else if (ch == '{' || ch == '[') {
      ++depth;
    } else if (ch == '}' || ch == ']') {
      if (--depth == 0) break;
    }
  }
  return out;
}

bool tuned_nd(const helm_ctx* c, TunedND& t) {
  const char* path = getenv("HELM_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  char key[128], rad[16] = "";
  if (c->r3 != 1) snprintf(rad, sizeof rad, ":r%d", c->r3);
  snprintf(key, sizeof key, "\"nd:%d:%dx%dx%d:%s%s\"", c->grid.dim, c->grid.n[0], c->grid.n[1],
           c->grid.dim == 3 ? c->grid.n[2] : 0, c->nd64 ? "f64" : "f32", rad);
  size_t k = txt.find(key);
  if (k == std::string::npos) return false;
  size_t ob = txt.find('{', k);
  if (ob == std::string::npos) return false;
  const std::map<std::string, std::string> m = json_members(txt, ob);
  auto num = [&](const char* name, int& out) {
    auto it = m.find(name);
    if (it != m.end()) out = atoi(it->second.c_str());
  };
  auto str = [&](const char* name, std::string& out, bool& has) {
    auto it = m.find(name);
    if (it != m.end()) {
      out = it->second;
      has = true;
    }
  };
  num("leaf", t.leaf);
  num("root", t.root);
  num("splitk_kb", t.splitk_kb);
  str("cuts", t.cuts, t.has_cuts);
  str("merge", t.merge, t.has_merge);
  str("boxes", t.boxes, t.has_boxes);
  return true;
}

std::vector<int> parse_cuts(const char* v) {
  std::vector<int> cuts;
  if (!strcmp(v, "none")) {
    cuts.push_back(-1);
    return cuts;
  }
  for (const char* p = v; *p;) {
    char* e = nullptr;
    long h = strtol(p, &e, 10);
    if (e == p) break;
    cuts.push_back((int)h);
    p = *e == ',' ? e + 1 : e;
  }
  return cuts;
}

// nested-dissection parameters: environment (HELM_ND_LEAF, HELM_ND_ROOT, HELM_ND_CUTS,
// HELM_ND_MERGE), else the autotuner's cache, else defaults and the planner's cost model
void build_plan(helm_ctx* c) {
  TunedND tn;
  const bool tuned = tuned_nd(c, tn);
  const int leaf = env_int("HELM_ND_LEAF", tuned && tn.leaf > 0 ? tn.leaf : (c->grid.dim == 3 ? 8 : 32));
  const int merge = env_int("HELM_ND_ROOT", tuned && tn.root > 0 ? tn.root : (c->grid.dim == 3 ? 1 : 1100));
  const int lds = env_int("HELM_ND_LDS", 65536);
  // cuts: heights closing the tree-block launches ("3,6,8"), "none" for none, empty for
  // the cost model's choice
  std::vector<int> cuts;
  if (const char* v = getenv("HELM_ND_CUTS"))
    cuts = parse_cuts(v);
  else if (tuned && tn.has_cuts)
    cuts = parse_cuts(tn.cuts.c_str());
  // merged heights: "1,3,5" (heights of the dissection tree whose fronts join their
  // parents), "none" or empty for none
  std::vector<int> mh;
  {
    const char* v = getenv("HELM_ND_MERGE");
    std::string mv = v ? std::string(v) : (tuned && tn.has_merge ? tn.merge : std::string());
    if (!mv.empty() && mv != "none") mh = parse_cuts(mv.c_str());
  }
  // box variants of the cycle kernels: "a,b,c,d" (HELM_BOXES, else the cache; default 0)
  {
    const char* v = getenv("HELM_BOXES");
    std::string bv = v ? std::string(v) : (tuned && tn.has_boxes ? tn.boxes : std::string());
    std::vector<int> bx = bv.empty() ? std::vector<int>() : parse_cuts(bv.c_str());
    for (int q = 0; q < 4; ++q) {
      c->box[q] = q < (int)bx.size() ? bx[q] : 0;
      const int nmax = (q % 2 == 0) ? 6 : 5;     // sweeps: 6 variants, restrictions: 5
      if (c->box[q] < 0 || c->box[q] >= nmax) throw std::runtime_error("HELM_BOXES: variant out of range");
    }
  }
  c->nd_merge = 0;
  for (int h : mh) {
    if (h < 0 || h > 62) throw std::runtime_error("HELM_ND_MERGE: heights 0..62");
    c->nd_merge |= 1LL << h;
  }
  c->tuned = tuned;
  c->nd_leaf = leaf;
  c->nd_root = merge;
  // heights above the tree blocks with at least this many factor bytes use split-K launches
  const long long splitk =
      (long long)env_int("HELM_ND_SPLITK_KB", tuned && tn.splitk_kb > 0 ? tn.splitk_kb : 4096) * 1024;
  // tree-block work-groups of at most HELM_ND_TREE_WAVES wavefronts: 16 in 2D; 8 in 3D, where
  // the many small subtrees run two work-groups per CU (measured 3 % faster at 256^3)
  const int tree_waves = env_int("HELM_ND_TREE_WAVES", c->grid.dim == 3 ? 8 : 16);
  nd_plan(c->g3, leaf, 16, merge, (int)c->ndsz, lds, cuts, splitk, c->plan, tree_waves, mh, c->r3);
  NDPlan& P = c->plan;
  c->hlist.clear();
  c->hlist_toff.clear();
  c->hinfo.clear();
  for (int h = 0; h <= P.max_height; ++h) {
    HeightInfo hi{};
    hi.start = (int)c->hlist.size();
    hi.count = (int)P.by_height[h].size();
    long long toff = 0;
    for (int t : P.by_height[h]) {
      const NDFrontDev& f = P.fronts[t];
      c->hlist.push_back(t);
      c->hlist_toff.push_back(toff);
      toff += (long long)ND_KB * f.nF;
      hi.max_asm = std::max(hi.max_asm, f.asm_cnt);
      hi.max_nS = std::max(hi.max_nS, f.nS);
      hi.max_nF = std::max(hi.max_nF, f.nF);
      int nbc = 0;
      hi.max_child = std::max(hi.max_child, f.nchild);
      for (int q = 0; q < f.nchild; ++q) nbc = std::max(nbc, P.fronts[P.children[f.child_off + q]].nB);
      hi.max_nb2 = std::max(hi.max_nb2, (long long)nbc * nbc);
      hi.max_T = std::max(hi.max_T, (long long)ND_KB * f.nF);
      hi.max_fin = std::max(hi.max_fin, (long long)f.nF * f.nS + (long long)f.nS * f.nB);
      hi.f_bytes += (long long)sizeof(cd) * f.nF * f.nF;
    }
    c->hinfo.push_back(hi);
  }
}

// the cycle's per-call scratch for rc right-hand sides, taken from cv (the sizes of the
// coarsest solve's buffers, d.*_n, must have been set)
CycleScratch carve_scratch(const helm_ctx* c, Carver& cv, int rc) {
  const size_t cs = c->csz, ns = c->ndsz, r = (size_t)rc;
  const NDDev& d = c->nd;
  CycleScratch w;
  w.x1a = cv.take<char>(r * cs * c->g1.tot);
  w.x1b = cv.take<char>(r * cs * c->g1.tot);
  w.b2 = cv.take<char>(r * cs * c->g2.tot);
  w.x2a = cv.take<char>(r * cs * c->g2.tot);
  w.x2b = cv.take<char>(r * cs * c->g2.tot);
  w.b3 = cv.take<char>(r * ns * c->g3.tot);       // the coarsest solve's vectors: its precision
  w.x3 = cv.take<char>(r * ns * c->g3.tot);
  w.upd = cv.take<char>(r * ns * std::max<long long>(1, c->plan.upd_total));
  w.gvec = d.gvec_n ? cv.take<char>(r * ns * d.gvec_n) : nullptr;
  w.part = cv.take<char>(r * ns * d.part_n);
  return w;
}

// carve every device buffer; returns the bytes used
size_t carve(helm_ctx* c, void* ws) {
  Carver cv(ws);
  const Geom &g1 = c->g1, &g2 = c->g2, &g3 = c->g3;
  const int m = c->mg.restart;
  const size_t cs = c->csz;
  NDPlan& P = c->plan;
  NDDev& d = c->nd;
  c->m64 = cv.take<double>(g1.tot);
  c->m32 = cv.take<float>(g1.tot);
  c->dg32 = c->f32 && !c->compact ? cv.take<cf>(g1.tot) : nullptr;
  c->coef2_64 = cv.take<cd>((size_t)c->K2 * g2.tot);
  // the 3D FP32 cycle keeps the complex-symmetric level-2 operator's centre and the 13
  // directions after it (14 of 27 planes); in 2D the mirrored reads cost more than the
  // 4 of 9 planes they save (measured), so all 9 are kept
  // (the compact stack's level-2 operator is not complex symmetric: all its planes are kept)
  c->coef2_32 = c->f32 ? cv.take<cf>((size_t)(c->compact ? c->K2 : sym2_planes(g2.dim)) * g2.tot) : nullptr;
  c->tmp2 = cv.take<cd>((size_t)c->K2 * g2.tot);
  c->coef3_64 = cv.take<cd>((size_t)c->K3 * g3.tot);
  const size_t rc = (size_t)c->rcap;
  c->r3d = cv.take<cd>(g3.tot);
  c->e3d = cv.take<cd>(g3.tot);
  // ND tables
  d.fronts = cv.take<NDFrontDev>(P.fronts.size());
  d.idx = cv.take<int>(P.idx.size());
  d.maps = cv.take<int>(std::max<size_t>(1, P.maps.size()));
  d.cptr = cv.take<int>(std::max<size_t>(1, P.cptr.size()));
  d.cidx = cv.take<int>(std::max<size_t>(1, P.cidx.size()));
  d.children = cv.take<int>(std::max<size_t>(1, P.children.size()));
  d.child_map_off = cv.take<long long>(std::max<size_t>(1, P.child_map_off.size()));
  {
    size_t mx = 1;
    size_t nc = 1;     // pivot candidates of the multi-work-group panels: fronts x row blocks of 32
    size_t pbr = 1;    // panel-buffer rows: fronts x rows rounded to 32, over the multi-panel heights
    // every height takes the multi-work-group panel when HELM_ND_LDS_PANEL is 0, else those
    // whose fronts are too large for the register panel (as nd_factor decides)
    const bool all_multi = getenv("HELM_ND_LDS_PANEL") && env_int("HELM_ND_LDS_PANEL", 0) <= 0;
    for (auto& h : P.by_height) {
      mx = std::max(mx, h.size());
      int mf = 0;
      for (int t : h) mf = std::max(mf, P.fronts[t].nF);
      const size_t rows = h.size() * (size_t)((mf + 31) / 32) * 32;
      nc = std::max(nc, rows / 32);
      if (all_multi || panel_reg_kb(mf) == 0) pbr = std::max(pbr, rows);
    }
    d.swp = cv.take<int>((size_t)ND_KBMAX * mx);
    d.cand = cv.take<PivCand>(2 * nc);
    d.pb = cv.take<cd>(pbr * ND_KBMAX);
  }
  d.asmv = cv.take<NDAsm>(P.asmv.size());
  d.perm = cv.take<int>(P.perm_total);
  d.hlist = cv.take<int>(c->hlist.size());
  d.hfr = cv.take<NDFrontDev>(c->hlist.size());   // the fronts in height order (factorisation)
  d.toff = cv.take<long long>(c->hlist_toff.size());
  d.err = cv.take<int>(1);
  d.F = cv.take<cd>(P.F_total);
  d.T = cv.take<cd>(std::max<long long>(1, P.T_scratch));
  d.L = cv.take<char>(c->ndsz * P.L_alloc);
  d.W = cv.take<char>(c->ndsz * std::max<long long>(1, P.W_alloc));
  long long part_max = 1;      // split-K partial products (entries)
  for (int fb = 0; fb < 2; ++fb) {
    std::vector<NDLaunch>& Ls = fb == 0 ? P.fwd : P.bwd;
    d.launch[fb].assign(Ls.size(), NDLaunchDev());
    for (size_t l = 0; l < Ls.size(); ++l) {
      const NDLaunch& L = Ls[l];
      NDLaunchDev& D = d.launch[fb][l];
      D.kind = L.kind;
      D.threads = L.threads;
      D.lds_bytes = L.lds_bytes;
      if (L.kind == 2) {
        D.ntasks = (int)L.tasks.size();
        D.tasks = cv.take<NDTask>(std::max<size_t>(1, L.tasks.size()));
        D.stages = cv.take<NDStage>(std::max<size_t>(1, L.stages.size()));
        D.gath = cv.take<NDGather>(std::max<size_t>(1, L.gath.size()));
        D.segs = cv.take<NDSeg>(std::max<size_t>(1, L.segs.size()));
        D.outs = cv.take<NDOut>(std::max<size_t>(1, L.outs.size()));
        D.dst = cv.take<int>(std::max<size_t>(1, L.dst.size()));
      } else if (L.kind == 3) {
        D.ngath = (int)L.gath.size();
        D.ntiles = (int)L.tiles.size();
        D.nrt = (int)L.rtiles.size();
        D.gath = cv.take<NDGather>(std::max<size_t>(1, L.gath.size()));
        D.tiles = cv.take<NDTile>(std::max<size_t>(1, L.tiles.size()));
        D.rtiles = cv.take<NDRowTile>(std::max<size_t>(1, L.rtiles.size()));
        part_max = std::max(part_max, L.p_elems);
      } else {
        D.ntasks = (int)L.task_off.size() - 1;
        D.task_off = cv.take<int>(L.task_off.size());
        D.items = cv.take<NDItem>(L.items.size());
        D.gath = cv.take<NDGather>(std::max<size_t>(1, L.gath.size()));
      }
    }
  }
  // global fall-back vectors for launches whose vectors do not fit in LDS
  // (a subtree task holds one vector per wavefront)
  long long gcap = 0, gneed = 0;
  for (int fb = 0; fb < 2; ++fb)
    for (size_t l = 0; l < (fb == 0 ? P.fwd : P.bwd).size(); ++l) {
      const NDLaunch& L = (fb == 0 ? P.fwd : P.bwd)[l];
      if (L.kind != 1) continue;
      const size_t need = (size_t)L.max_rows_vec * c->ndsz;
      d.launch[fb][l].shm = need <= c->lds_limit ? std::max<size_t>(need, 16) : 0;
      // 1024-thread work-groups (64 k-splits) where a vector exceeds 256 entries, if the
      // launch fits the chip at once (decided at launch time with the right-hand sides)
      d.launch[fb][l].threads = L.max_rows_vec > 256 ? 1024 : 256;
      if (need > c->lds_limit) {
        gcap = std::max<long long>(gcap, L.max_rows_vec);
        gneed = std::max<long long>(gneed, (long long)(L.task_off.size() - 1));
      }
    }
  d.gvec_cap = (int)gcap;
  d.gvec_n = gcap * gneed;
  d.part_n = part_max;
  c->scr = carve_scratch(c, cv, (int)rc);
  // Krylov
  c->V = cv.take<cd>(rc * (m + 1) * g1.tot);
  c->Z = cv.take<char>(rc * cs * (size_t)m * g1.tot);
  long long nblk = (g1.tot + 256 * KNPT - 1) / (256 * KNPT);
  c->part = cv.take<cd>(rc * (2 * KMAXM + 3) * nblk);
  c->st = cv.take<KrylovState>(rc);
  c->Bm = rc > 1 ? cv.take<cd>(rc * g1.tot) : nullptr;
  c->Xm = rc > 1 ? cv.take<cd>(rc * g1.tot) : nullptr;
  return cv.off;
}

template <typename T>
void up(T* dst, const std::vector<T>& v, hipStream_t s) {
  if (!v.empty()) CK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

cd shift_scalar(double alpha, double beta, double omega) {
  // alpha^2 (1 - i beta) omega^2
  double w2 = omega * omega * alpha * alpha;
  return mk(w2, -beta * w2);
}

void nd_factor(helm_ctx* c, hipStream_t s) {
  NDDev& d = c->nd;
  NDPlan& P = c->plan;
  nd_zero(d.F, P.F_total, s);
  nd_iota(d.perm, d.fronts, (int)P.fronts.size(), s);
  CK(hipMemsetAsync(d.err, 0, sizeof(int), s));
  for (size_t h = 0; h < c->hinfo.size(); ++h) {
    const HeightInfo& hi = c->hinfo[h];
    const int* ids = d.hlist + hi.start;
    const NDFrontDev* hf = d.hfr + hi.start;     // the height's fronts, slot order
    const long long* toff = d.toff + hi.start;
    nd_assemble(d.fronts, ids, hi.count, hi.max_asm, d.asmv, c->coef3_64, d.F, s);
    for (int slot = 0; slot < hi.max_child; ++slot)
      nd_extend(d.fronts, ids, hi.count, hi.max_nb2, d.children, d.child_map_off, d.maps, d.F, slot, s);
    // the register-resident panel (one work-group per front) when the fronts are small
    // enough; otherwise the panel is spread over many work-groups
    const int kreg = panel_reg_kb(hi.max_nF);
    const bool reg_panel = kreg > 0 && c->lds_panel > 0;
    // multi-work-group panels: HELM_ND_KB_MULTI columns (16, 32 or 64).  Every pivot step
    // reads and writes its panel over all rows of the front, so with the trailing passes
    // taken per block the narrower 32-column panel is the faster one.
    // Panels are grouped into blocks of HELM_ND_KB_OUTER columns: the panels of a block
    // update each other, and the rest of the front takes one trailing update per block, so
    // the GEMM streams the front once per block instead of once per panel.  For the 8- to
    // 32-column register panels that pass is bound by the fronts' traffic, and blocking
    // pays once the height's fronts hold at least HELM_ND_REG_BLOCK_MB megabytes and have
    // at least two blocks' worth of rows; below that every pass costs about one launch (and
    // a block covers most of a small front), so the block's two extra launches do not pay.
    const int kmulti = std::max(8, std::min(ND_KBMAX, env_int("HELM_ND_KB_MULTI", 32)));
    const int kb = reg_panel ? kreg : kmulti;
    const int reg_mb = env_int("HELM_ND_REG_BLOCK_MB", 32);
    const bool blocked = !reg_panel || (hi.f_bytes >= (long long)reg_mb * 1000000 &&
                                        (reg_mb == 0 || hi.max_nF >= 2 * ND_KBOUT));
    const int kout = blocked ? std::max(1, std::min(ND_KBOUT, env_int("HELM_ND_KB_OUTER", ND_KBOUT)) / kb) * kb : kb;
    for (int k0 = 0; k0 < hi.max_nS; k0 += kout) {
      for (int k1 = k0; k1 < std::min(k0 + kout, hi.max_nS); k1 += kb) {
        if (reg_panel)
          nd_panel_reg(hf, nullptr, hi.count, hi.max_nF, d.F, d.perm, d.swp, k1, kb, d.err, s);
        else
          nd_panel_multi(hf, hi.count, hi.max_nF, d.F, d.pb, d.perm, d.swp, d.cand, k1, kb, hi.max_nS, d.err, s);
        if (kout > kb) {        // the block's other panels, earlier ones included
          nd_save_t(hf, nullptr, hi.count, toff, (long long)kb * kout, d.F, d.T, k1, kb, k0, kout, s);
          nd_gemm(hf, nullptr, hi.count, toff, hi.max_nF, kout, d.F, d.T, k1, kb, k0, kout, s);
        }
      }
      nd_save_t(hf, nullptr, hi.count, toff, hi.max_T, d.F, d.T, k0, kout, 0, -1, s);
      nd_gemm(hf, nullptr, hi.count, toff, hi.max_nF, hi.max_nF, d.F, d.T, k0, kout, 0, -1, s);
    }
    if (!c->nd64)
      nd_finalize<cf>(hf, nullptr, hi.count, hi.max_fin, d.F, d.perm, (cf*)d.L, (cf*)d.W, s);
    else
      nd_finalize<cd>(hf, nullptr, hi.count, hi.max_fin, d.F, d.perm, (cd*)d.L, (cd*)d.W, s);
  }
}

hipEvent_t ev_get(helm_ctx* c) {
  if (!c->evpool.empty()) {
    hipEvent_t e = c->evpool.back();
    c->evpool.pop_back();
    return e;
  }
  hipEvent_t e;
  CK(hipEventCreate(&e));
  return e;
}
// resolve recorded event pairs (the stream must have been synchronised)
void ev_flush(helm_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0;
    CK(hipEventElapsedTime(&ms, p.a, p.b));
    c->kt_ms[p.cls] += ms;
    c->kt_cnt[p.cls] += p.launches;
    c->evpool.push_back(p.a);
    c->evpool.push_back(p.b);
  }
  c->pending.clear();
}
#define TIMED(c, cls, s, stmt)                                  \
  do {                                                          \
    hipEvent_t a_ = nullptr;                                    \
    if ((c)->timing) {                                          \
      a_ = ev_get(c);                                           \
      CK(hipEventRecord(a_, s));                                \
    }                                                           \
    stmt;                                                       \
    if ((c)->timing) {                                          \
      hipEvent_t b_ = ev_get(c);                                \
      CK(hipEventRecord(b_, s));                                \
      (c)->pending.push_back(Pending{cls, a_, b_, 1});          \
    }                                                           \
  } while (0)

template <typename C>
void nd_solve(helm_ctx* c, const CycleScratch& w, const C* r, C* x, int conj, hipStream_t s) {
  NDDev& d = c->nd;
  NDRhs rh;
  rh.n = c->nr;
  rh.vec = c->g3.tot;
  rh.upd = std::max<long long>(1, c->plan.upd_total);
  rh.part = d.part_n;
  rh.gvec = d.gvec_n;
  // timing: one event pair around each direction's launches (they run back to back), so
  // that the per-launch average carries no per-launch event overhead
  hipEvent_t e0 = nullptr;
  if (c->timing) CK(hipEventRecord(e0 = ev_get(c), s));
  for (const NDLaunchDev& L : d.launch[0]) {
    C* gv = L.kind == 1 && L.shm == 0 ? (C*)w.gvec : nullptr;
    nd_fwd<C>(L, d.fronts, d.idx, d.cptr, d.cidx, (const C*)d.L, (C*)w.upd, r, x, gv, d.gvec_cap, conj,
              (C*)w.part, rh, s);
  }
  hipEvent_t e1 = nullptr;
  if (c->timing) {
    CK(hipEventRecord(e1 = ev_get(c), s));
    c->pending.push_back(Pending{KT_ND_FWD, e0, e1, nd_kernels(d.launch[0])});
  }
  for (const NDLaunchDev& L : d.launch[1]) {
    C* gv = L.kind == 1 && L.shm == 0 ? (C*)w.gvec : nullptr;
    nd_bwd<C>(L, d.fronts, d.idx, d.cidx, (const C*)d.W, (C*)w.upd, x, gv, d.gvec_cap, conj, (C*)w.part,
              rh, s);
  }
  if (c->timing && !d.launch[1].empty()) {
    hipEvent_t e2 = ev_get(c);
    CK(hipEventRecord(e2, s));
    c->pending.push_back(Pending{KT_ND_BWD, e1, e2, nd_kernels(d.launch[1])});
  }
}


// a0-a3: coefficients, Galerkin operators, real-shifted coarsest operator, factorisation.
// medium: the slowness kappa (is_m = 0) or its square m (is_m = 1) at every node
void numeric_setup(helm_ctx* c, const double* medium, int is_m, hipStream_t s) {
  const helm_shift* shift = &c->shift;
  const double omega = c->omega;
  // a0: m = kappa^2 (FP64 and FP32); the FP32 cycle's level-1 diagonal
  square_slowness(medium, c->m64, c->m32, c->g1.tot, is_m, s);
  if (c->compact) {
    // the compact stack: A2 = R1 H_beta^{alpha2} P1, A3 = R2 (R1 H_beta^alpha P1) P2 with
    // its transfers (eqs. 2.2, 3.3-3.6), then the exact factorisation
    wgal_fine(c->op, shift_scalar(shift->alpha2, shift->beta, omega), c->m64, c->g2, c->tr[0], c->ip[0], c->r2,
              c->coef2_64, s);
    if (c->f32) cast_d2f(c->coef2_64, c->coef2_32, (long long)c->K2 * c->g2.tot, s);
    wgal_fine(c->op, shift_scalar(shift->alpha, shift->beta, omega), c->m64, c->g2, c->tr[0], c->ip[0], c->r2,
              c->tmp2, s);
    wgal_coarse(c->g2, c->tmp2, c->r2, c->g3, c->tr[1], c->ip[1], c->r3, c->coef3_64, s);
    nd_factor(c, s);
    return;
  }
  if (c->f32) {
    L1<float> A;
    A.op = c->op;
    const cd sb = shift_scalar(1.0, shift->beta, omega);
    A.s = mk((float)sb.x, (float)sb.y);
    A.m = c->m32;
    A.conj = 0;
    l1_diag32(A, c->dg32, s);
  }
  // a1: level-2 Galerkin operator of H_beta^{alpha2}
  gal_fine(c->op, shift_scalar(shift->alpha2, shift->beta, omega), c->m64, c->g2, c->coef2_64, s);
  const int K = stencil_points(c->grid.dim);
  if (c->f32)
    cast_d2f(c->coef2_64 + (long long)(K - sym2_planes(c->g2.dim)) * c->g2.tot, c->coef2_32,
             (long long)sym2_planes(c->g2.dim) * c->g2.tot, s);
  // a2: real-shifted level-3 operator R2 (R1 H_beta^alpha P1) P2
  gal_fine(c->op, shift_scalar(shift->alpha, shift->beta, omega), c->m64, c->g2, c->tmp2, s);
  gal_coarse(c->g2, c->tmp2, c->g3, c->coef3_64, s);
  // a3: exact factorisation
  nd_factor(c, s);
}

// iterate state of one level: x_in = [x] + [w D^-1 b] + [P e]
template <typename C>
struct St {
  int xin;
  C* x;
};

template <typename R>
struct Cycle {
  typedef typename cplx<R>::type C;
  helm_ctx* c;
  int conj;
  hipStream_t s;
  CycleScratch w;       // where the iterates and the coarsest solve's buffers live
  L1<R> A1;
  L2<R> A2;

  Cycle(helm_ctx* ctx, int op, hipStream_t st) : Cycle(ctx, op, st, ctx->scr) {}
  Cycle(helm_ctx* ctx, int op, hipStream_t st, const CycleScratch& scr) : c(ctx), conj(op), s(st), w(scr) {
    A1.op = c->op;
    cd sb = shift_scalar(1.0, c->shift.beta, c->omega);
    A1.s = mk((R)sb.x, (R)sb.y);
    A1.m = (const R*)(sizeof(R) == 4 ? (const void*)c->m32 : (const void*)c->m64);
    A1.conj = op;
    A1.dg = (const C*)(sizeof(R) == 4 ? (const void*)c->dg32 : nullptr);
    A1.box_sweep = c->box[0];
    A1.box_restrict = c->box[1];
    A2.g = c->g2;
    A2.coef = (const C*)(sizeof(R) == 4 ? (const void*)c->coef2_32 : (const void*)c->coef2_64);
    A2.conj = op;
    A2.box_sweep = c->box[2];
    A2.box_restrict = c->box[3];
  }

  // level 1: one more sweep (or the virtual first sweep) on state st
  template <typename CO>
  St<C> adv1(St<C> st, const cd* b, const C* e, CO* out) {
    R w = (R)c->mg.jacobi[0];
    TIMED(c, KT_L1_SWEEP, s, (l1_sweep<R, cd, CO>(A1, st.xin, st.x, b, w, c->g2, e, w, out, c->nr, s)));
    return St<C>{XIN_X, (C*)out};
  }
  St<C> adv2(St<C> st, const C* b, const C* e, C* out) {
    R w = (R)c->mg.jacobi[1];
    TIMED(c, KT_L2_SWEEP, s, (l2_sweep<R>(A2, st.xin, st.x, b, w, c->g3, e, w, out, c->nr, s)));
    return St<C>{XIN_X, out};
  }
  C* other(C* cur, C* a, C* b) { return cur == a ? b : a; }

  // the compact stack's cycle (the two-grid algorithm of Sec. 2 applied recursively, in
  // the order of the oracle's cycle): plain Jacobi sweeps, residuals and transfers, the
  // level-2 visits continuing from the current level-2 iterate (x2 + cycle(b2 - A2 x2)
  // equals the visit from a zero guess on the updated residual).  nullptr iterates are zero.
  template <typename CO>
  void run_wide(const cd* b1, CO* out) {
    const helm_mg& mg = c->mg;
    const int nr = c->nr;
    C *x1a = (C*)w.x1a, *x1b = (C*)w.x1b, *x2a = (C*)w.x2a, *x2b = (C*)w.x2b;
    C* b2 = (C*)w.b2;
    const R w1 = (R)mg.jacobi[0], w2 = (R)mg.jacobi[1];
    WFine<R> F;
    F.op = c->op;
    const cd sb = shift_scalar(1.0, c->shift.beta, c->omega);
    F.s = mk((R)sb.x, (R)sb.y);
    F.m = (const R*)(sizeof(R) == 4 ? (const void*)c->m32 : (const void*)c->m64);
    const C* A2c = (const C*)(sizeof(R) == 4 ? (const void*)c->coef2_32 : (const void*)c->coef2_64);
    auto free1 = [&](const C* x) { return x == x1a ? x1b : x1a; };
    auto free2 = [&](const C* x) { return x == x2a ? x2b : x2a; };
    // level 1: pre-relaxation, residual, restriction
    C* x1 = nullptr;
    for (int k = 0; k < mg.nu_pre; ++k) {
      C* o = free1(x1);
      TIMED(c, KT_L1_SWEEP, s, (w1_step<R, cd, C>(F, WM_JAC, x1 == nullptr, x1, b1, w1, o, nr, s)));
      x1 = o;
    }
    C* r1 = free1(x1);
    TIMED(c, KT_L1_RESTRICT, s, (w1_step<R, cd, C>(F, WM_RES, x1 == nullptr, x1, b1, (R)0, r1, nr, s)));
    TIMED(c, KT_L1_RESTRICT, s, (w_restrict<C, C>(c->g1, r1, c->g2, c->tr[0], b2, nr, s)));
    // level 2: gamma visits
    C* x2 = nullptr;
    for (int v = 0; v < mg.cycle; ++v) {
      for (int k = 0; k < mg.nu_pre; ++k) {
        C* o = free2(x2);
        TIMED(c, KT_L2_SWEEP, s, (w2_step<R>(c->g2, A2c, c->r2, WM_JAC, x2 == nullptr, x2, b2, w2, o, nr, s)));
        x2 = o;
      }
      C* r2 = free2(x2);
      TIMED(c, KT_L2_RESTRICT, s, (w2_step<R>(c->g2, A2c, c->r2, WM_RES, x2 == nullptr, x2, b2, (R)0, r2, nr, s)));
      // the coarsest solve in its own precision (FP64 for this stack)
      if (c->nd64) {
        TIMED(c, KT_L2_RESTRICT, s, (w_restrict<C, cd>(c->g2, r2, c->g3, c->tr[1], (cd*)w.b3, nr, s)));
        nd_solve<cd>(c, w, (const cd*)w.b3, (cd*)w.x3, 0, s);
      } else {
        TIMED(c, KT_L2_RESTRICT, s, (w_restrict<C, cf>(c->g2, r2, c->g3, c->tr[1], (cf*)w.b3, nr, s)));
        nd_solve<cf>(c, w, (const cf*)w.b3, (cf*)w.x3, 0, s);
      }
      const int add = x2 != nullptr;
      if (x2 == nullptr) x2 = r2;   // a zero iterate: x2 = P2 x3
      if (c->nd64)
        w_prolong<cd, C>(c->g3, (const cd*)w.x3, c->g2, c->ip[1], add, x2, nr, s);
      else
        w_prolong<cf, C>(c->g3, (const cf*)w.x3, c->g2, c->ip[1], add, x2, nr, s);
      for (int k = 0; k < mg.nu_post; ++k) {
        C* o = free2(x2);
        TIMED(c, KT_L2_SWEEP, s, (w2_step<R>(c->g2, A2c, c->r2, WM_JAC, 0, x2, b2, w2, o, nr, s)));
        x2 = o;
      }
    }
    // level 1: correction and post-relaxation; the last sweep writes `out`
    if (x1 == nullptr) {
      x1 = x1a;
      w_prolong<C, C>(c->g2, x2, c->g1, c->ip[0], 0, x1, nr, s);
    } else {
      w_prolong<C, C>(c->g2, x2, c->g1, c->ip[0], 1, x1, nr, s);
    }
    if (mg.nu_post == 0) {
      w_copy<C, CO>(x1, out, (long long)nr * c->g1.tot, s);
      return;
    }
    for (int k = 0; k < mg.nu_post; ++k) {
      if (k == mg.nu_post - 1) {
        TIMED(c, KT_L1_SWEEP, s, (w1_step<R, cd, CO>(F, WM_JAC, 0, x1, b1, w1, out, nr, s)));
      } else {
        C* o = free1(x1);
        TIMED(c, KT_L1_SWEEP, s, (w1_step<R, cd, C>(F, WM_JAC, 0, x1, b1, w1, o, nr, s)));
        x1 = o;
      }
    }
  }

  template <typename CO>
  void run(const cd* b1, CO* out) {
    if (c->compact) {
      run_wide<CO>(b1, out);
      return;
    }
    const helm_mg& mg = c->mg;
    C *x1a = (C*)w.x1a, *x1b = (C*)w.x1b, *x2a = (C*)w.x2a, *x2b = (C*)w.x2b;
    C *b2 = (C*)w.b2, *b3 = (C*)w.b3, *x3 = (C*)w.x3;
    R w1 = (R)mg.jacobi[0], w2 = (R)mg.jacobi[1];
    // ---- level 1 pre-relaxation
    St<C> s1{0, nullptr};
    for (int k = 0; k < mg.nu_pre; ++k) {
      if (s1.xin == 0) s1 = St<C>{XIN_Z, nullptr};
      else s1 = adv1<C>(s1, b1, nullptr, other(s1.x, x1a, x1b));
    }
    TIMED(c, KT_L1_RESTRICT, s,
          (l1_restrict<R, cd>(A1, s1.xin, s1.x, b1, w1, c->g2, nullptr, c->g2, b2, c->nr, s)));
    // ---- level 2 visits.  In 2D with one pre- and one post-sweep, the post-sweep of a
    // visit, the pre-sweep of the next and its restriction run as one kernel (l2_chain)
    St<C> s2{0, nullptr};
    const bool chain = c->l2_chain && c->g2.dim == 2 && mg.nu_pre == 1 && mg.nu_post == 1;
    // in 2D with one pre- and one post-sweep, the last level-2 post-sweep and the level-1
    // post-sweep run as one kernel (cycle_tail)
    const bool tail = chain && s1.xin == XIN_Z;
    bool chained = false;       // this visit's pre-sweep and restriction are done
    for (int v = 0; v < mg.cycle; ++v) {
      if (!chained) {
        for (int k = 0; k < mg.nu_pre; ++k) {
          if (s2.xin == 0) s2 = St<C>{XIN_Z, nullptr};
          else s2 = adv2(s2, b2, nullptr, other(s2.x, x2a, x2b));
        }
        TIMED(c, KT_L2_RESTRICT, s,
              (l2_restrict<R>(A2, s2.xin, s2.x, b2, w2, c->g3, nullptr, c->g3, b3, c->nr, s)));
      }
      nd_solve<C>(c, w, b3, x3, conj, s);
      s2.xin |= XIN_E;
      // the last visit's post-sweep, left to the cycle's tail (below)
      if (tail && v + 1 == mg.cycle && s2.xin == (XIN_X | XIN_E)) break;
      chained = chain && v + 1 < mg.cycle && s2.xin == (XIN_Z | XIN_E);
      if (chained) {
        C* xb = other(s2.x, x2a, x2b);
        TIMED(c, KT_L2_CHAIN, s, (l2_chain<R>(A2, s2.xin, s2.x, b2, w2, c->g3, x3, w2, xb, b3, c->nr, s)));
        s2 = St<C>{XIN_X, xb};
        continue;
      }
      for (int k = 0; k < mg.nu_post; ++k) s2 = adv2(s2, b2, x3, other(s2.x, x2a, x2b));
      if (s2.xin != XIN_X) {   // materialise (no post-relaxation)
        R w0 = 0;
        l2_sweep<R>(A2, s2.xin, s2.x, b2, w2, c->g3, x3, w0, other(s2.x, x2a, x2b), c->nr, s);
        s2 = St<C>{XIN_X, other(s2.x, x2a, x2b)};
      }
    }
    // ---- level 1 correction and post-relaxation; the last sweep writes `out`
    if (tail && s2.xin == (XIN_X | XIN_E)) {
      TIMED(c, KT_TAIL, s, (cycle_tail<R, CO>(A1, b1, w1, A2, s2.x, b2, w2, c->g3, x3, out, c->nr, s)));
      return;
    }
    s1.xin |= XIN_E;
    const C* e2 = s2.x;
    if (mg.nu_post == 0) {
      l1_sweep<R, cd, CO>(A1, s1.xin, s1.x, b1, w1, c->g2, e2, (R)0, out, c->nr, s);
      return;
    }
    for (int k = 0; k < mg.nu_post; ++k) {
      if (k == mg.nu_post - 1)
        adv1<CO>(s1, b1, e2, out);
      else
        s1 = adv1<C>(s1, b1, e2, other(s1.x, x1a, x1b));
    }
  }
};

// the scalar block of KrylovState, as read back by the host
struct HostScalars {
  double bnorm, beta0, est, hnext, true_rel;
  int its, done, final, nonfinite, kcols, maxit;
};
static_assert(sizeof(HostScalars) == offsetof(KrylovState, hist) - offsetof(KrylovState, bnorm),
              "HostScalars must mirror the scalar block of KrylovState");
constexpr size_t HSLOT = 1024;   // bytes between the slots of hstate (16 right-hand sides)
constexpr int RMAX = (int)(HSLOT / sizeof(HostScalars));
inline HostScalars* hs(helm_ctx* c, int slot = 0) { return (HostScalars*)(c->hstate + HSLOT * slot); }
// the scalar blocks of the nr states into slot `slot` of hstate (asynchronous: one small
// kernel writes them into the pinned buffer through its device mapping)
void read_states_async(helm_ctx* c, int slot, hipStream_t s) {
  KrylovArgs a;
  a.st = c->st;
  a.nrhs = c->nr;
  kr_pack_states(a, c->hstate_dev + HSLOT * slot, s);
}
void read_states(helm_ctx* c, hipStream_t s) {
  read_states_async(c, 0, s);
  CK(hipStreamSynchronize(s));
}

KrylovArgs make_kargs(helm_ctx* c, int op) {
  KrylovArgs a;
  a.op = c->op;
  a.s = mk(c->omega * c->omega, 0.0);
  a.conj = op;
  a.m64 = c->m64;
  a.V = c->V;
  a.ldv = (long long)c->nr * c->g1.tot;
  a.part = c->part;
  a.nblk = (int)((c->g1.tot + 256 * KNPT - 1) / (256 * KNPT));
  a.pcap = a.nblk;
  a.st = c->st;
  a.nrhs = c->nr;
  a.pstride = (long long)(2 * KMAXM + 3) * a.pcap;
  a.guard = c->arnoldi_guard;
  return a;
}

void drop_graphs(helm_ctx* c) {
  for (int op = 0; op < 2; ++op) {
    for (hipGraphExec_t g : c->gexec[op]) (void)hipGraphExecDestroy(g);
    c->gexec[op].clear();
    c->gtol[op] = -1.0;
  }
}

// capture and instantiation are serialised over the process: batched solves run one host
// worker per stream, and the HIP runtime's capture bookkeeping is not relied on to be
// safe for concurrent captures from several threads
std::mutex g_capture_mu;

// capture the m per-iteration graphs of operator op for the current right-hand side count
// (kernel arguments are fixed: buffers, shifts, tolerance), once per context until the
// frequency, the shifts or the count change
template <typename R>
void iter_graphs(helm_ctx* c, int op, double tol) {
  typedef typename cplx<R>::type C;
  const int m = c->mg.restart;
  if ((int)c->gexec[op].size() == m && c->gtol[op] == tol && c->gnr[op] == c->nr) return;
  std::lock_guard<std::mutex> lock(g_capture_mu);
  for (hipGraphExec_t g : c->gexec[op]) (void)hipGraphExecDestroy(g);
  c->gexec[op].clear();
  if (!c->cap) CK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  KrylovArgs a = make_kargs(c, op);
  Cycle<R> cyc(c, op, c->cap);
  const size_t NJ = (size_t)c->nr * c->g1.tot;    // entries between basis vectors
  const int saved = c->timing;
  c->timing = 0;
  for (int j = 0; j < m; ++j) {
    hipGraph_t g = nullptr;
    CK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    cyc.template run<C>(c->V + j * NJ, (C*)c->Z + j * NJ);
    // the state read-back of this position into its slot of the pinned buffer is made by
    // the update pass inside the graph: a separate launch between graphs cost a dispatch
    // and about 8 us of idle device, one inside it about 4 us
    kr_arnoldi(a, (const char*)c->Z + j * NJ * c->csz, c->f32, j, tol, c->hstate_dev + HSLOT * (1 + (j & 1)),
               c->tail_fused, c->cap);
    CK(hipStreamEndCapture(c->cap, &g));
    hipGraphExec_t e = nullptr;
    CK(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    c->gexec[op].push_back(e);
  }
  c->timing = saved;
  c->gtol[op] = tol;
  c->gnr[op] = c->nr;
}

// FGMRES(m) on nr right-hand sides in lock-step: b, x hold right-hand side r at r N1.
// Each has its own Krylov state; one that has converged (or stopped) keeps its state
// done, and its Krylov kernels do nothing.  info: nr entries (or NULL).
template <typename R>
int solve_impl(helm_ctx* c, int op, int nr, const cd* b, cd* x, double tol, int max_iter, helm_solve_info* info,
               hipStream_t s) {
  c->nr = nr;
  KrylovArgs a = make_kargs(c, op);
  Cycle<R> cyc(c, op, s);
  typedef typename cplx<R>::type C;
  const int m = c->mg.restart;
  const long long N = c->g1.tot;
  const size_t NJ = (size_t)nr * N;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    CK(hipEventRecord(e0, s));
  }
  const bool use_graphs = c->graphs && !c->timing;
  if (use_graphs) iter_graphs<R>(c, op, tol);
  kr_init(a, max_iter, s);
  kr_residual(a, x, b, 1, s);
  read_states(c, s);
  std::vector<int> status(nr, HELM_OK), its(nr, 0), restarts(nr, 0), kc(nr, 0);
  std::vector<double> est(nr, 0.0), true_rel(nr, 0.0), prev_rel(nr, 0.0);
  std::vector<char> fin(nr, 0);
  unsigned newly = 0;
  for (int r = 0; r < nr; ++r) {
    const HostScalars& h = hs(c)[r];
    if (!std::isfinite(h.bnorm) || !std::isfinite(h.beta0)) {
      status[r] = HELM_ENONFINITE;
      fin[r] = 1;
    } else if (h.bnorm == 0.0) {
      kr_zero(x + r * N, N, s);
      fin[r] = 1;
    } else {
      true_rel[r] = est[r] = prev_rel[r] = h.beta0 / h.bnorm;
      if (true_rel[r] <= tol) fin[r] = 1;
    }
    if (fin[r]) newly |= 1u << r;
  }
  if (newly) kr_finalize(a, newly, s);
  auto active = [&]() {
    for (int r = 0; r < nr; ++r)
      if (!fin[r]) return true;
    return false;
  };
  // every unfinished right-hand side's column is done (converged, stopped or non-finite)
  auto all_done = [&](const HostScalars* h) {
    for (int r = 0; r < nr; ++r)
      if (!fin[r] && !h[r].done && !h[r].nonfinite) return false;
    return true;
  };
  while (active()) {
    kr_scale_v0(a, s);
    if (use_graphs) {
      // iteration q + 1 is queued before the states of iteration q are read back, so the
      // device does not wait for the host between iterations.  An iteration queued after
      // a right-hand side's last one finds its done flag set: its Krylov kernels return at
      // once and leave its basis, Hessenberg column and counters as they are.
      auto queue = [&](int j) {
        CK(hipGraphLaunch(c->gexec[op][j], s));
        // (the graph ends with the read-back of its states into slot 1 + (j & 1))
        CK(hipEventRecord(c->itev[j & 1], s));
      };
      for (hipEvent_t& e : c->itev)
        if (!e) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      int q = 0, k = 0;          // iterations of this cycle queued, read
      queue(q++);
      while (k < q) {
        if (q < m) queue(q++);
        CK(hipEventSynchronize(c->itev[k & 1]));
        std::memcpy(hs(c), hs(c, 1 + (k & 1)), sizeof(HostScalars) * nr);
        ++k;
        if (all_done(hs(c))) break;
      }
    } else {
      for (int j = 0; j < m; ++j) {
        if (c->timing) kr_hold(150, s);     // the iteration's launches are queued before they run
        cyc.template run<C>(c->V + j * NJ, (C*)c->Z + j * NJ);
        TIMED(c, KT_APPLY_DOT, s, kr_arnoldi(a, (const char*)c->Z + j * NJ * c->csz, c->f32, j, tol,
                                             c->hstate_dev, c->tail_fused, s));
        CK(hipStreamSynchronize(s));
        if (all_done(hs(c))) break;
      }
    }
    for (int r = 0; r < nr; ++r)
      if (!fin[r]) {
        const HostScalars& h = hs(c)[r];
        its[r] = h.its;
        est[r] = h.est;
        kc[r] = h.kcols;
        if (h.nonfinite) {
          status[r] = HELM_ENONFINITE;
          fin[r] = 2;           // finished with no update of x
        }
      }
    kr_update_x(a, c->Z, c->f32, (long long)NJ, x, s);
    kr_residual(a, x, b, 0, s);
    read_states(c, s);
    newly = 0;
    for (int r = 0; r < nr; ++r) {
      if (fin[r] == 2) {
        fin[r] = 1;
        newly |= 1u << r;
        continue;
      }
      if (fin[r]) continue;
      const HostScalars& h = hs(c)[r];
      true_rel[r] = h.beta0 / h.bnorm;
      if (!std::isfinite(true_rel[r])) {
        status[r] = HELM_ENONFINITE;
        fin[r] = 1;
      } else if (true_rel[r] <= tol) {
        fin[r] = 1;
      } else if (its[r] >= max_iter) {
        status[r] = HELM_ENOCONV;
        fin[r] = 1;
      } else if (kc[r] == m && true_rel[r] >= prev_rel[r] * (1.0 - 1e-12)) {
        status[r] = HELM_ESTAGNATE;
        fin[r] = 1;
      } else {
        prev_rel[r] = true_rel[r];
        ++restarts[r];
      }
      if (fin[r]) newly |= 1u << r;
    }
    if (newly) kr_finalize(a, newly, s);
  }
  if (c->timing) {
    CK(hipEventRecord(e1, s));
    CK(hipEventSynchronize(e1));
    float ms = 0;
    CK(hipEventElapsedTime(&ms, e0, e1));
    c->times[0] = ms;
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
  }
  CK(hipStreamSynchronize(s));
  ev_flush(c);
  int worst = HELM_OK;
  for (int r = 0; r < nr; ++r) {
    if (info) {
      helm_solve_info& I = info[r];
      I.iterations = its[r];
      I.restarts = restarts[r];
      I.status = status[r];
      I.est_rel_residual = est[r];
      I.true_rel_residual = true_rel[r];
      if (I.history && I.history_cap > 0 && its[r] > 0) {
        int n = std::min(std::min(its[r], I.history_cap), KMAXIT);
        CK(hipMemcpy(I.history, (char*)(c->st + r) + offsetof(KrylovState, hist), n * sizeof(double),
                     hipMemcpyDeviceToHost));
      }
    }
    if (status[r] < 0 && worst >= 0) worst = status[r];
    else if (worst >= 0) worst = std::max(worst, status[r]);
  }
  return worst;
}

// The cycle as a stand-alone solver (the stationary iteration x <- x + M^{-1}(b - op(H) x),
// the paper's use of the method "as a solver"): one cycle, the update and the FP64 residual
// per iteration, the host reading the residual norm after each.  info->history receives the
// relative residual after every cycle.  A residual that grows beyond 1e8 ||b|| ends the
// iteration (HELM_ENOCONV).
template <typename R>
int stationary_impl(helm_ctx* c, int op, const cd* b, cd* x, double tol, int max_iter, helm_solve_info* info,
                    hipStream_t s) {
  typedef typename cplx<R>::type C;
  c->nr = 1;
  KrylovArgs a = make_kargs(c, op);
  Cycle<R> cyc(c, op, s);
  const long long N = c->g1.tot;
  kr_init(a, max_iter, s);
  kr_residual(a, x, b, 1, s);         // V_0 = b - op(H) x, ||b||, ||V_0||
  read_states(c, s);
  const double bnorm = hs(c)->bnorm;
  double rel = hs(c)->beta0 / bnorm;
  int status = HELM_OK, its = 0;
  std::vector<double> hist;
  if (!std::isfinite(bnorm) || !std::isfinite(hs(c)->beta0)) {
    status = HELM_ENONFINITE;
  } else if (bnorm == 0.0) {
    kr_zero(x, N, s);
    rel = 0.0;
  } else {
    while (rel > tol && its < max_iter) {
      cyc.template run<C>(c->V, (C*)c->Z);           // z = M^{-1} r
      kr_add_z(a, c->Z, c->f32, x, s);               // x += z
      kr_residual(a, x, b, 0, s);                    // r = b - op(H) x, in FP64
      read_states(c, s);
      ++its;
      rel = hs(c)->beta0 / bnorm;
      hist.push_back(rel);
      if (!std::isfinite(rel)) {
        status = HELM_ENONFINITE;
        break;
      }
      if (rel > 1e8) break;
    }
    if (status == HELM_OK && rel > tol) status = HELM_ENOCONV;
  }
  CK(hipStreamSynchronize(s));
  ev_flush(c);
  if (info) {
    info->iterations = its;
    info->restarts = 0;
    info->status = status;
    info->est_rel_residual = rel;
    info->true_rel_residual = rel;
    if (info->history && info->history_cap > 0)
      for (int k = 0; k < std::min(its, info->history_cap); ++k) info->history[k] = hist[k];
  }
  return status;
}

}  // namespace

// =========================================================================== C ABI
extern "C" {

const char* helm_status_str(int st) {
  switch (st) {
    case HELM_OK: return "ok";
    case HELM_EINVAL: return "invalid argument";
    case HELM_EWORKSPACE: return "workspace missing, misaligned or too small";
    case HELM_EDEVICE: return "device error";
    case HELM_ENONFINITE: return "non-finite value";
    case HELM_ESINGULAR: return "zero pivot in the coarsest-grid elimination";
    case HELM_ENOCONV: return "not converged within max_iter";
    case HELM_ESTAGNATE: return "stagnated over a full restart cycle";
    default: return "unknown status";
  }
}

const char* helm_last_error(void) { return g_err; }

// rcap: right-hand sides a context solves in lock-step (its buffers are carved for them)
static int ws_bytes_rcap(const helm_grid* grid, const helm_mg* mg, int rcap, size_t* bytes) {
  int v = validate(grid, mg);
  if (v) return v;
  if (!bytes) return fail(HELM_EINVAL, "bytes is NULL");
  try {
    helm_ctx c;
    c.grid = *grid;
    c.mg = *mg;
    c.rcap = rcap;
    init_geometry(&c);
    build_plan(&c);
    *bytes = carve(&c, nullptr);
    return HELM_OK;
  } catch (std::exception& e) {
    return fail(HELM_EINVAL, "%s", e.what());
  }
}

int helm_workspace_bytes(const helm_grid* grid, const helm_mg* mg, size_t* bytes) {
  return ws_bytes_rcap(grid, mg, 1, bytes);
}

static int setup_rcap(const helm_grid* grid, const double* slowness, double omega, const helm_shift* shift,
                      const helm_mg* mg, int rcap, void* ws, size_t ws_bytes, void* stream, helm_ctx** out) {
  int v = validate(grid, mg);
  if (v) return v;
  if (!slowness || !shift || !out) return fail(HELM_EINVAL, "NULL slowness/shift/out");
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(HELM_EINVAL, "omega must be positive and finite");
  if (!std::isfinite(shift->alpha) || !std::isfinite(shift->alpha2) || !std::isfinite(shift->beta))
    return fail(HELM_EINVAL, "shift parameters must be finite");
  if (!ws || ((uintptr_t)ws % ALIGN) != 0) return fail(HELM_EWORKSPACE, "workspace NULL or not 256-byte aligned");
  *out = nullptr;
  std::unique_ptr<helm_ctx> c(new helm_ctx());
  hipStream_t s = (hipStream_t)stream;
  try {
    c->grid = *grid;
    c->mg = *mg;
    c->shift = *shift;
    c->omega = omega;
    c->rcap = rcap;
    c->graphs = env_int("HELM_GRAPHS", 1);
    c->l2_chain = env_int("HELM_L2_CHAIN", 1);
    // HELM_ARNOLDI_GUARD (tests): the cancellation threshold of the Arnoldi norm formula
    if (const char* g = getenv("HELM_ARNOLDI_GUARD")) c->arnoldi_guard = atof(g);
    init_geometry(c.get());
    build_plan(c.get());
    size_t need = carve(c.get(), nullptr);
    if (ws_bytes < need) return fail(HELM_EWORKSPACE, "workspace too small: %zu < %zu", ws_bytes, need);
    c->ws_needed = need;
    carve(c.get(), ws);
    CK(hipHostMalloc((void**)&c->hstate, 4096, hipHostMallocMapped | hipHostMallocCoherent));
    CK(hipHostGetDevicePointer((void**)&c->hstate_dev, c->hstate, 0));
    {
      int dev = 0, lds = 0;
      CK(hipGetDevice(&dev));
      CK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      c->lds_panel = lds > 4096 ? (size_t)lds - 2048 : 0;
      // HELM_ND_LDS_PANEL caps the LDS-resident panel (bytes; 0: every panel takes the
      // multi-work-group path)
      if (getenv("HELM_ND_LDS_PANEL")) c->lds_panel = std::min<size_t>(c->lds_panel, (size_t)env_int("HELM_ND_LDS_PANEL", 0));
      if (env_int("HELM_VERBOSE", 0)) fprintf(stderr, "helm: LDS per block %d bytes\n", lds);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    CK(hipEventRecord(e0, s));
    // tables
    NDPlan& P = c->plan;
    NDDev& d = c->nd;
    up(d.fronts, P.fronts, s);
    up(d.idx, P.idx, s);
    up(d.maps, P.maps, s);
    up(d.cptr, P.cptr, s);
    up(d.cidx, P.cidx, s);
    up(d.children, P.children, s);
    up(d.child_map_off, P.child_map_off, s);
    up(d.asmv, P.asmv, s);
    up(d.hlist, c->hlist, s);
    {
      std::vector<NDFrontDev> hf;
      hf.reserve(c->hlist.size());
      for (int t : c->hlist) hf.push_back(P.fronts[t]);
      up(d.hfr, hf, s);
    }
    up(d.toff, c->hlist_toff, s);
    for (int fb = 0; fb < 2; ++fb) {
      std::vector<NDLaunch>& Ls = fb == 0 ? P.fwd : P.bwd;
      for (size_t l = 0; l < Ls.size(); ++l) {
        NDLaunchDev& D = d.launch[fb][l];
        if (Ls[l].kind == 2) {
          up((NDTask*)D.tasks, Ls[l].tasks, s);
          up((NDStage*)D.stages, Ls[l].stages, s);
          up((NDGather*)D.gath, Ls[l].gath, s);
          up((NDSeg*)D.segs, Ls[l].segs, s);
          up((NDOut*)D.outs, Ls[l].outs, s);
          up((int*)D.dst, Ls[l].dst, s);
        } else if (Ls[l].kind == 3) {
          up((NDGather*)D.gath, Ls[l].gath, s);
          up((NDTile*)D.tiles, Ls[l].tiles, s);
          up((NDRowTile*)D.rtiles, Ls[l].rtiles, s);
        } else {
          up((int*)D.task_off, Ls[l].task_off, s);
          up((NDItem*)D.items, Ls[l].items, s);
          up((NDGather*)D.gath, Ls[l].gath, s);
        }
      }
    }
    numeric_setup(c.get(), slowness, 0, s);
    CK(hipEventRecord(e1, s));
    CK(hipStreamSynchronize(s));
    CK(hipGetLastError());
    float ms = 0;
    CK(hipEventElapsedTime(&ms, e0, e1));
    c->times[4] = ms;
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    int err = 0;
    CK(hipMemcpy(&err, d.err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
      (void)hipHostFree(c->hstate);
      return fail(HELM_ESINGULAR, "zero pivot in the coarsest-grid elimination");
    }
  } catch (DevErr& e) {
    if (c->hstate) (void)hipHostFree(c->hstate);
    return fail(HELM_EDEVICE, "%s", e.what());
  } catch (std::exception& e) {
    if (c->hstate) (void)hipHostFree(c->hstate);
    return fail(HELM_EINVAL, "%s", e.what());
  }
  *out = c.release();
  return HELM_OK;
}

int helm_setup(const helm_grid* grid, const double* slowness, double omega, const helm_shift* shift,
               const helm_mg* mg, void* ws, size_t ws_bytes, void* stream, helm_ctx** out) {
  return setup_rcap(grid, slowness, omega, shift, mg, 1, ws, ws_bytes, stream, out);
}

static int refactor_impl(helm_ctx* c, const double* medium, int is_m, double omega, const helm_shift* shift,
                         void* stream) {
  if (!c || !medium || !shift) return fail(HELM_EINVAL, "NULL argument");
  if (int v = need_single(c, "helm_refactor")) return v;
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(HELM_EINVAL, "omega must be positive and finite");
  if (!std::isfinite(shift->alpha) || !std::isfinite(shift->alpha2) || !std::isfinite(shift->beta))
    return fail(HELM_EINVAL, "shift parameters must be finite");
  hipStream_t s = (hipStream_t)stream;
  try {
    if (omega != c->omega || shift->alpha != c->shift.alpha || shift->alpha2 != c->shift.alpha2 ||
        shift->beta != c->shift.beta)
      drop_graphs(c);          // captured kernel arguments hold the shifted coefficients' scalars
    c->omega = omega;
    c->shift = *shift;
    numeric_setup(c, medium, is_m, s);
    int err = 0;
    CK(hipMemcpyAsync(c->hstate, c->nd.err, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    std::memcpy(&err, c->hstate, sizeof(int));
    if (err) return fail(HELM_ESINGULAR, "zero pivot in the coarsest-grid elimination");
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  return HELM_OK;
}

int helm_refactor(helm_ctx* c, const double* slowness, double omega, const helm_shift* shift, void* stream) {
  return refactor_impl(c, slowness, 0, omega, shift, stream);
}

int helm_refactor_m(helm_ctx* c, const double* m, double omega, const helm_shift* shift, void* stream) {
  return refactor_impl(c, m, 1, omega, shift, stream);
}

int helm_destroy(helm_ctx* ctx) {
  if (!ctx) return HELM_OK;
  for (helm_ctx* q : ctx->sub) helm_destroy(q);
  drop_graphs(ctx);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  for (hipStream_t t : ctx->bstreams) (void)hipStreamDestroy(t);
  if (ctx->hstate) (void)hipHostFree(ctx->hstate);
  for (hipEvent_t e : ctx->itev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
  delete ctx;
  return HELM_OK;
}

int helm_apply(helm_ctx* c, int op, int prec, const void* x, void* y, void* stream) {
  if (!c || !x || !y) return fail(HELM_EINVAL, "NULL argument");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (prec != HELM_F64 && prec != HELM_F32) return fail(HELM_EINVAL, "prec must be HELM_F64 or HELM_F32");
  if (x == y) return fail(HELM_EINVAL, "x and y must differ");
  if (int v = need_single(c, "helm_apply")) return v;
  if (int v = need_op(c, op, "helm_apply")) return v;
  hipStream_t s = (hipStream_t)stream;
  try {
    if (c->compact) {
      if (prec == HELM_F64) {
        WFine<double> F;
        F.op = c->op;
        F.s = mk(c->omega * c->omega, 0.0);
        F.m = c->m64;
        w1_step<double, cd, cd>(F, WM_APPLY, 0, (const cd*)x, (const cd*)nullptr, 0.0, (cd*)y, 1, s);
      } else {
        WFine<float> F;
        F.op = c->op;
        F.s = mk((float)(c->omega * c->omega), 0.f);
        F.m = c->m32;
        w1_step<float, cf, cf>(F, WM_APPLY, 0, (const cf*)x, (const cf*)nullptr, 0.f, (cf*)y, 1, s);
      }
    } else if (prec == HELM_F64) {
      L1<double> A;
      A.op = c->op;
      A.s = mk(c->omega * c->omega, 0.0);
      A.m = c->m64;
      A.conj = op;
      l1_apply64(A, x, 0, (cd*)y, s);
    } else {
      L1<float> A;
      A.op = c->op;
      A.s = mk((float)(c->omega * c->omega), 0.f);
      A.m = c->m32;
      A.conj = op;
      l1_apply32(A, (const cf*)x, (cf*)y, s);
    }
    CK(hipGetLastError());
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  return HELM_OK;
}

int helm_vcycle(helm_ctx* c, int op, const void* r, void* z, void* stream) {
  if (!c || !r || !z) return fail(HELM_EINVAL, "NULL argument");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (r == z) return fail(HELM_EINVAL, "r and z must differ");
  if (int v = need_single(c, "helm_vcycle")) return v;
  if (int v = need_op(c, op, "helm_vcycle")) return v;
  hipStream_t s = (hipStream_t)stream;
  c->nr = 1;
  try {
    if (c->f32) {
      Cycle<float> cyc(c, op, s);
      cyc.template run<cd>((const cd*)r, (cd*)z);
    } else {
      Cycle<double> cyc(c, op, s);
      cyc.template run<cd>((const cd*)r, (cd*)z);
    }
    CK(hipGetLastError());
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  return HELM_OK;
}

int helm_coarse_solve(helm_ctx* c, int op, const void* r, void* e, void* stream) {
  if (!c || !r || !e) return fail(HELM_EINVAL, "NULL argument");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (r == e) return fail(HELM_EINVAL, "r and e must differ");
  if (int v = need_single(c, "helm_coarse_solve")) return v;
  if (int v = need_op(c, op, "helm_coarse_solve")) return v;
  hipStream_t s = (hipStream_t)stream;
  c->nr = 1;
  try {
    if (!c->nd64) {
      cast_d2f((const cd*)r, (cf*)c->scr.b3, c->g3.tot, s);
      nd_solve<cf>(c, c->scr, (const cf*)c->scr.b3, (cf*)c->scr.x3, op, s);
      cast_f2d((const cf*)c->scr.x3, (cd*)e, c->g3.tot, s);
    } else {
      nd_solve<cd>(c, c->scr, (const cd*)r, (cd*)e, op, s);
    }
    CK(hipGetLastError());
  } catch (DevErr& ex) {
    return fail(HELM_EDEVICE, "%s", ex.what());
  }
  return HELM_OK;
}

int helm_solve(helm_ctx* c, int op, const void* rhs, void* x, double tol, int max_iter, helm_solve_info* info,
               void* stream) {
  if (!c || !rhs || !x) return fail(HELM_EINVAL, "NULL argument");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HELM_EINVAL, "tol must be positive");
  if (max_iter < 1) return fail(HELM_EINVAL, "max_iter must be >= 1");
  if (rhs == x) return fail(HELM_EINVAL, "rhs and x must differ");
  if (int v = need_single(c, "helm_solve")) return v;
  if (int v = need_op(c, op, "helm_solve")) return v;
  hipStream_t s = (hipStream_t)stream;
  try {
    int st = c->f32 ? solve_impl<float>(c, op, 1, (const cd*)rhs, (cd*)x, tol, max_iter, info, s)
                    : solve_impl<double>(c, op, 1, (const cd*)rhs, (cd*)x, tol, max_iter, info, s);
    CK(hipGetLastError());
    return st;
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
}

int helm_iterate(helm_ctx* c, int op, const void* rhs, void* x, double tol, int max_iter, helm_solve_info* info,
                 void* stream) {
  if (!c || !rhs || !x) return fail(HELM_EINVAL, "NULL argument");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HELM_EINVAL, "tol must be positive");
  if (max_iter < 1) return fail(HELM_EINVAL, "max_iter must be >= 1");
  if (rhs == x) return fail(HELM_EINVAL, "rhs and x must differ");
  if (int v = need_single(c, "helm_iterate")) return v;
  if (int v = need_op(c, op, "helm_iterate")) return v;
  hipStream_t s = (hipStream_t)stream;
  try {
    int st = c->f32 ? stationary_impl<float>(c, op, (const cd*)rhs, (cd*)x, tol, max_iter, info, s)
                    : stationary_impl<double>(c, op, (const cd*)rhs, (cd*)x, tol, max_iter, info, s);
    CK(hipGetLastError());
    return st;
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
}

int helm_set_timing(helm_ctx* c, int on) {
  if (!c) return fail(HELM_EINVAL, "NULL context");
  c->timing = on ? 1 : 0;
  for (int k = 0; k < KT_N; ++k) {
    c->kt_ms[k] = 0.0;
    c->kt_cnt[k] = 0;
  }
  for (helm_ctx* u : c->sub) helm_set_timing(u, on);
  return HELM_OK;
}

int helm_get_timing(helm_ctx* c, double* t, int n) {
  if (!c || !t || n < 0) return fail(HELM_EINVAL, "bad arguments");
  try {
    ev_flush(c);
    for (helm_ctx* u : c->sub) ev_flush(u);
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  std::vector<double> v(c->times, c->times + 5);
  for (int k = 0; k < KT_N; ++k) {
    double ms = c->kt_ms[k], cnt = (double)c->kt_cnt[k];
    for (helm_ctx* u : c->sub) {           // batched: the sums over the instances
      ms += u->kt_ms[k];
      cnt += (double)u->kt_cnt[k];
    }
    v.push_back(ms);
    v.push_back(cnt);
  }
  int m = std::min<int>(n, (int)v.size());
  for (int i = 0; i < m; ++i) t[i] = v[i];
  return m;
}

int helm_get_info(helm_ctx* c, long long* out, int n) {
  if (!c || !out || n < 0) return fail(HELM_EINVAL, "bad arguments");
  if (!c->sub.empty()) return fail(HELM_EINVAL, "single-instance contexts only");
  const NDPlan& P = c->plan;
  long long sB = 0, maxF = 0;
  for (const NDFrontDev& f : P.fronts) {
    sB += f.nB;
    maxF = std::max<long long>(maxF, f.nF);
  }
  long long v[29] = {c->g1.tot, c->g2.tot, c->g3.tot, (long long)P.fronts.size(), P.L_total, P.W_total, sB,
                     c->g3.tot, (long long)nd_kernels(c->nd.launch[0]), (long long)nd_kernels(c->nd.launch[1]),
                     (long long)c->ws_needed, maxF,
                     (long long)c->csz, c->nd_leaf, c->nd_root, c->tuned ? 1 : 0, (long long)P.cuts.size(),
                     -1, -1, -1, -1, c->nd_merge, c->K2, c->K3, (long long)c->ndsz,
                     c->box[0], c->box[1], c->box[2], c->box[3]};
  for (size_t i = 0; i < P.cuts.size() && i < 4; ++i) v[17 + i] = P.cuts[i];
  int m = std::min(n, 29);
  for (int i = 0; i < m; ++i) out[i] = v[i];
  return m;
}

int helm_get_instance_info(helm_ctx* c, int inst, long long* out, int n) {
  if (!c) return fail(HELM_EINVAL, "NULL context");
  if (c->sub.empty()) {
    if (inst != 0) return fail(HELM_EINVAL, "instance %d of a single-instance context", inst);
    return helm_get_info(c, out, n);
  }
  if (inst < 0 || inst >= (int)c->sub.size()) return fail(HELM_EINVAL, "no instance %d", inst);
  return helm_get_info(c->sub[inst], out, n);
}

long long helm_level_size(helm_ctx* c, int inst, int lev) {
  if (!c) return -1;
  if (!c->sub.empty()) {
    if (inst < 0 || inst >= (int)c->sub.size()) return -1;
    c = c->sub[inst];
  } else if (inst != 0) {
    return -1;
  }
  if (lev == 1) return c->g1.tot;
  if (lev == 2) return c->g2.tot;
  if (lev == 3) return c->g3.tot;
  return -1;
}

int helm_get_coefficients(helm_ctx* c, int lev, double* out) {
  if (!c || !out) return fail(HELM_EINVAL, "NULL argument");
  if (lev != 2 && lev != 3) return fail(HELM_EINVAL, "lev must be 2 or 3");
  if (int v = need_single(c, "helm_get_coefficients")) return v;
  try {
    const Geom& g = lev == 2 ? c->g2 : c->g3;
    const cd* src = lev == 2 ? c->coef2_64 : c->coef3_64;
    CK(hipDeviceSynchronize());
    CK(hipMemcpy(out, src, sizeof(cd) * (lev == 2 ? c->K2 : c->K3) * g.tot, hipMemcpyDeviceToHost));
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  return HELM_OK;
}

int helm_grad_m(helm_ctx* c, int n_src, const void* const* u, const void* const* lambda, double* g, int accumulate,
                void* stream) {
  if (!c || !u || !lambda || !g || n_src < 1) return fail(HELM_EINVAL, "bad arguments");
  for (int k = 0; k < n_src; ++k)
    if (!u[k] || !lambda[k]) return fail(HELM_EINVAL, "NULL source pointer %d", k);
  if (int v = need_single(c, "helm_grad_m")) return v;
  if (c->compact)
    return fail(HELM_EINVAL, "helm_grad_m: the compact stack has no adjoint path (its H is not complex symmetric)");
  hipStream_t s = (hipStream_t)stream;
  try {
    for (int k = 0; k < n_src; ++k)
      grad_accumulate(c->op, c->omega, (const cd*)u[k], (const cd*)lambda[k], g, (k == 0 && !accumulate),
                      s);
    CK(hipGetLastError());
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  return HELM_OK;
}

}  // extern "C"

// =========================================================================== batched form
// A batched context owns one single-instance context per instance, carved from
// consecutive slices of the caller's workspace; right-hand sides are solved with
// their instance's hierarchy.
extern "C" {

// right-hand sides per instance solved in lock-step (at most RMAX)
static int batch_rcap(int max_rhs) { return std::max(1, std::min(max_rhs, RMAX)); }

int helm_workspace_bytes_batched(int n_inst, const helm_grid* grids, const helm_mg* mg, int max_rhs,
                                 size_t* bytes) {
  if (n_inst < 1 || !grids || !mg || !bytes || max_rhs < 1) return fail(HELM_EINVAL, "bad arguments");
  size_t tot = 0;
  for (int i = 0; i < n_inst; ++i) {
    size_t b = 0;
    int v = ws_bytes_rcap(&grids[i], mg, batch_rcap(max_rhs), &b);
    if (v) return v;
    tot += al(b);
  }
  *bytes = tot;
  return HELM_OK;
}

int helm_workspace_bytes_multi(const helm_grid* grid, const helm_mg* mg, int max_rhs, size_t* bytes) {
  if (!grid || !mg || !bytes || max_rhs < 1) return fail(HELM_EINVAL, "bad arguments");
  return ws_bytes_rcap(grid, mg, batch_rcap(max_rhs), bytes);
}

int helm_setup_multi(const helm_grid* grid, const double* slowness, double omega, const helm_shift* shift,
                     const helm_mg* mg, int max_rhs, void* ws, size_t ws_bytes, void* stream, helm_ctx** out) {
  if (max_rhs < 1) return fail(HELM_EINVAL, "max_rhs must be >= 1");
  return setup_rcap(grid, slowness, omega, shift, mg, batch_rcap(max_rhs), ws, ws_bytes, stream, out);
}

int helm_setup_batched(int n_inst, const helm_grid* grids, const double* const* slowness, const double* omega,
                       const helm_shift* shift, const helm_mg* mg, int max_rhs, void* ws, size_t ws_bytes,
                       void* stream, helm_ctx** out) {
  if (n_inst < 1 || !grids || !slowness || !omega || !shift || !mg || !out || max_rhs < 1)
    return fail(HELM_EINVAL, "bad arguments");
  size_t need = 0;
  int v = helm_workspace_bytes_batched(n_inst, grids, mg, max_rhs, &need);
  if (v) return v;
  if (!ws || ((uintptr_t)ws % ALIGN) != 0 || ws_bytes < need)
    return fail(HELM_EWORKSPACE, "workspace NULL, misaligned or too small (%zu < %zu)", ws_bytes, need);
  *out = nullptr;
  const int rcap = batch_rcap(max_rhs);
  std::unique_ptr<helm_ctx> b(new helm_ctx());
  b->grid = grids[0];
  b->mg = *mg;
  char* p = (char*)ws;
  for (int i = 0; i < n_inst; ++i) {
    size_t bi = 0;
    ws_bytes_rcap(&grids[i], mg, rcap, &bi);
    helm_ctx* c = nullptr;
    int r = setup_rcap(&grids[i], slowness[i], omega[i], &shift[i], mg, rcap, p, al(bi), stream, &c);
    if (r) {
      for (helm_ctx* q : b->sub) helm_destroy(q);
      return r;
    }
    // instances are solved concurrently on several streams: there the fences of the fused
    // FGMRES tail write back L2 lines that the other streams' kernels use (2.4 % fewer
    // solves per second on the 96-instance workload), so their final sums and Givens step
    // are separate launches;
    // and the device is busy, so the fused level-2 chain and cycle tail, which save
    // launches at the cost of halo work, measured 2 % fewer solves per second there
    c->tail_fused = n_inst == 1;
    if (n_inst > 1) c->l2_chain = 0;
    b->sub.push_back(c);
    p += al(bi);
  }
  *out = b.release();
  return HELM_OK;
}

int helm_solve_batched(helm_ctx* ctx, int op, int n_rhs, const int* inst_of_rhs, const void* const* rhs,
                       void* const* x, double tol, int max_iter, helm_solve_info* info, void* stream) {
  if (!ctx || n_rhs < 1 || !inst_of_rhs || !rhs || !x) return fail(HELM_EINVAL, "bad arguments");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HELM_EINVAL, "tol must be positive");
  if (max_iter < 1) return fail(HELM_EINVAL, "max_iter must be >= 1");
  if (int v = need_op(ctx->sub.empty() ? ctx : ctx->sub[0], op, "helm_solve_batched")) return v;
  const int ninst = ctx->sub.empty() ? 1 : (int)ctx->sub.size();
  std::vector<std::vector<int>> by(ninst);      // right-hand sides of each instance, in order
  for (int k = 0; k < n_rhs; ++k) {
    if (inst_of_rhs[k] < 0 || inst_of_rhs[k] >= ninst || !rhs[k] || !x[k] || rhs[k] == x[k])
      return fail(HELM_EINVAL, "bad right-hand side %d", k);
    by[inst_of_rhs[k]].push_back(k);
  }
  std::vector<int> busy;
  for (int i = 0; i < ninst; ++i)
    if (!by[i].empty()) busy.push_back(i);
  hipStream_t s = (hipStream_t)stream;
  // instances are independent: they run concurrently on library-owned streams (one host
  // worker per stream); an instance's right-hand sides are solved in lock-step groups of
  // up to its capacity, one group after the other on its stream.  Workers take the next
  // instance when they finish one, larger grids first, so that the short solves fill in
  // at the end.
  std::stable_sort(busy.begin(), busy.end(), [&](int a, int b) {
    const long long na = ctx->sub.empty() ? ctx->g1.tot : ctx->sub[a]->g1.tot;
    const long long nb = ctx->sub.empty() ? ctx->g1.tot : ctx->sub[b]->g1.tot;
    return na > nb;
  });
  std::atomic<size_t> next_inst{0};
  std::vector<char> taken(busy.size(), 0);
  const int nst = std::max(1, std::min(env_int("HELM_BATCH_STREAMS", 8), (int)busy.size()));
  std::vector<int> status(n_rhs, HELM_OK);
  std::vector<std::string> errs(nst);
  try {
    while ((int)ctx->bstreams.size() < nst) {
      hipStream_t t;
      CK(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
      ctx->bstreams.push_back(t);
    }
    hipEvent_t ready;
    CK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    CK(hipEventRecord(ready, s));
    for (int w = 0; w < nst; ++w) CK(hipStreamWaitEvent(ctx->bstreams[w], ready, 0));
    // a new host thread starts on device 0: the workers take the caller's device
    int dev = 0;
    CK(hipGetDevice(&dev));
    std::vector<std::thread> pool;
    for (int w = 0; w < nst; ++w)
      pool.emplace_back([&, w]() {
        const hipStream_t sw = ctx->bstreams[w];
        if (hipSetDevice(dev) != hipSuccess) {
          errs[w] = "hipSetDevice failed in a batch worker";
          return;
        }
        for (;;) {
          const size_t q = next_inst.fetch_add(1);
          if (q >= busy.size()) break;
          taken[q] = 1;
          const int i = busy[q];
          helm_ctx* c = ctx->sub.empty() ? ctx : ctx->sub[i];
          const std::vector<int>& ks = by[i];
          if (c->rcap == 1) {
            for (int k : ks) {
              status[k] = helm_solve(c, op, rhs[k], x[k], tol, max_iter, info ? &info[k] : nullptr, sw);
              if (status[k] < 0) {
                errs[w] = helm_last_error();
                return;
              }
            }
            continue;
          }
          const long long N = c->g1.tot;
          const size_t vb = sizeof(cd) * (size_t)N;
          for (size_t t0 = 0; t0 < ks.size(); t0 += c->rcap) {
            const int nr = (int)std::min<size_t>(c->rcap, ks.size() - t0);
            helm_solve_info tmp[RMAX];
            try {
              for (int t = 0; t < nr; ++t) {
                const int k = ks[t0 + t];
                tmp[t] = helm_solve_info{};
                if (info) {
                  tmp[t].history = info[k].history;
                  tmp[t].history_cap = info[k].history_cap;
                }
                CK(hipMemcpyAsync(c->Bm + t * N, rhs[k], vb, hipMemcpyDeviceToDevice, sw));
                CK(hipMemcpyAsync(c->Xm + t * N, x[k], vb, hipMemcpyDeviceToDevice, sw));
              }
              if (c->f32)
                solve_impl<float>(c, op, nr, c->Bm, c->Xm, tol, max_iter, tmp, sw);
              else
                solve_impl<double>(c, op, nr, c->Bm, c->Xm, tol, max_iter, tmp, sw);
              for (int t = 0; t < nr; ++t)
                CK(hipMemcpyAsync(x[ks[t0 + t]], c->Xm + t * N, vb, hipMemcpyDeviceToDevice, sw));
              CK(hipStreamSynchronize(sw));
            } catch (DevErr& e) {
              errs[w] = e.what();
              for (int t = 0; t < nr; ++t) status[ks[t0 + t]] = HELM_EDEVICE;
              return;
            }
            for (int t = 0; t < nr; ++t) {
              const int k = ks[t0 + t];
              status[k] = tmp[t].status;
              if (info) info[k] = tmp[t];
            }
          }
        }
      });
    for (auto& t : pool) t.join();
    for (size_t q = 0; q < busy.size(); ++q)      // left over by workers that could not start
      if (!taken[q])
        for (int k : by[busy[q]]) status[k] = HELM_EDEVICE;
    for (int w = 0; w < nst; ++w) {
      CK(hipEventRecord(ready, ctx->bstreams[w]));
      CK(hipStreamWaitEvent(s, ready, 0));
    }
    CK(hipEventDestroy(ready));
  } catch (DevErr& e) {
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  int worst = HELM_OK;
  for (int k = 0; k < n_rhs; ++k) {
    if (status[k] < 0) {
      for (auto& e : errs)
        if (!e.empty()) return fail(status[k], "%s", e.c_str());
      return status[k];
    }
    worst = std::max(worst, status[k]);
  }
  return worst;
}

}  // extern "C"

// =========================================================================== cycle without allocation
// helm_vcycle_noalloc takes the cycle's per-call scratch from a fixed device array instead of
// the context's workspace, for callers that cannot allocate.  Every device the library runs
// on holds its own copy of the array from the library's load until the process ends.  In
// host code `scratch` names a host-side stand-in: its device address on the current device
// comes from hipGetSymbolAddress, resolved once per device and kept in g_scratch.
static __device__ __align__(256) char scratch[HELM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[SCRATCH_MAX_DEVICES] = {nullptr};

// the array's address on the current device (resolved on the first call on that device)
void* scratch_on_current_device() {
  int dev = 0;
  CK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) throw DevErr("device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    CK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr % ALIGN) != 0) throw DevErr("scratch array has no aligned device address");
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}
}  // namespace

extern "C" {

int helm_vcycle_noalloc(helm_ctx* c, int op, const void* r, void* z, void* stream) {
  if (!c || !r || !z) return fail(HELM_EINVAL, "NULL argument");
  if (op != HELM_OP_N && op != HELM_OP_C) return fail(HELM_EINVAL, "op must be HELM_OP_N or HELM_OP_C");
  if (r == z) return fail(HELM_EINVAL, "r and z must differ");
  if (int v = need_single(c, "helm_vcycle_noalloc")) return v;
  if (int v = need_op(c, op, "helm_vcycle_noalloc")) return v;
  size_t need = 0;
  {
    Carver probe(nullptr);
    carve_scratch(c, probe, 1);
    need = probe.off;
  }
  if (need > HELM_NOALLOC_SCRATCH_BYTES)
    return fail(HELM_EINVAL, "helm_vcycle_noalloc: this grid needs %zu bytes of scratch, the static array holds %zu",
                need, (size_t)HELM_NOALLOC_SCRATCH_BYTES);
  hipStream_t s = (hipStream_t)stream;
  const int saved_timing = c->timing;
  try {
    Carver cv(scratch_on_current_device());
    const CycleScratch w = carve_scratch(c, cv, 1);
    c->nr = 1;
    c->timing = 0;            // timing would create events
    if (c->f32) {
      Cycle<float> cyc(c, op, s, w);
      cyc.template run<cd>((const cd*)r, (cd*)z);
    } else {
      Cycle<double> cyc(c, op, s, w);
      cyc.template run<cd>((const cd*)r, (cd*)z);
    }
    c->timing = saved_timing;
    CK(hipGetLastError());
  } catch (DevErr& e) {
    c->timing = saved_timing;
    return fail(HELM_EDEVICE, "%s", e.what());
  }
  return HELM_OK;
}

}  // extern "C"
