// C-ABI and host driver of the MI355X randomized Krylov-Schur solver.
//
// rks_solve runs Algorithm 1: the first extension (Algorithm 2 from one
// column), then cycles of contraction (real Schur form of the active block,
// reordering of the wanted Ritz values to the front, truncation: the
// contraction of Algorithm 1), residual estimates (Section 4.1), locking (Section 4.4),
// optional whitening (Section 3.3), the basis rotation on the device and a
// new extension.  Each cycle crosses the host/device boundary once: the
// Rayleigh quotient B and the sketch S (both FP64, at most a few hundred KB)
// come to the host, the rotation Y and the truncated B, S go back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dense.h"
#include "launch.hpp"
#include "panels.hpp"
#include "rks.h"

using rks::cplx;

namespace {

constexpr double kUnitRoundoff = 0x1.0p-53;
constexpr double kBreakdownRel = 1e-12;

const char* code_str(int c) {
  switch (c) {
    case RKS_OK: return "ok";
    case RKS_ENOTCONV: return "not converged within max_restarts";
    case RKS_EINVAL: return "invalid argument";
    case RKS_ENOMEM: return "out of memory";
    case RKS_EHIP: return "HIP runtime error";
    case RKS_ENAN: return "non-finite value";
    case RKS_ESTATE: return "call order violated";
    case RKS_EBREAKDOWN: return "breakdown: exact invariant subspace";
    case RKS_EDENSE: return "small dense step failed";
    default: return "unknown error";
  }
}

struct EvPair {
  int cat;
  hipEvent_t a, b;
};

}  // namespace

struct rks_ctx {
  int64_t n = 0, nnz = 0;
  int k = 0, m = 0, d = 0, which = 0;
  double tol = 0.0;
  rks_opts o{};
  double normA1 = 0.0;
  rks::LaunchEnv env{};
  int vbytes = 8, wbytes = 8;  // bytes between rows of a basis column (the pair basis: its FP32 part), of w
  int ebytes = 8;              // HBM bytes of one basis element (the pair basis: 4 + 2)
  bool pair = false;           // pair basis (FP32 + 16-bit remainder)
  int64_t ldu = 0;
  // device buffers
  int *rp = nullptr, *col = nullptr, *tiles = nullptr, *flags = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  uint8_t* vidx = nullptr;  // value-indexed A (FP64 product): one byte per nonzero
  double* vtab = nullptr;   // its table of distinct values (256 entries)
  int a_distinct = 0;       // distinct values in vtab (0: FP64 values)
  // sliced layout (when chosen): slice offsets, columns and values in slice order
  int64_t* sl_off = nullptr;
  int* col_sl = nullptr;
  double* val_sl = nullptr;
  uint8_t* vidx_sl = nullptr;
  float* val32_sl = nullptr;
  void* U = nullptr;      // basis in use (U_lo or U64)
  void* U_lo = nullptr;   // basis in the requested precision (allocated at create; the pair
                          // basis: the FP32 parts, then the 16-bit remainders of the same elements)
  double* xcur = nullptr; // pair basis: FP64 copy of the column written last (ldu values)
  void* U64 = nullptr;    // FP64 basis of the refinement phase (lazy)
  void* w = nullptr;
  double phase_tol = 0.0;
  double *S = nullptr, *B = nullptr, *cs = nullptr, *coef = nullptr, *z = nullptr, *sr = nullptr;
  double *zpart = nullptr, *spart = nullptr, *scal = nullptr, *Yd = nullptr, *u0tmp = nullptr;
  double* E = nullptr;  // S^T S - I, (m+1) x (m+1), leading dimension m+1
  double* kpart = nullptr;  // deterministic Krylov-Schur: partial rows of U^T x (kMaxG x (m+1))
  bool ks = false;          // deterministic Krylov-Schur (RKS_METHOD_KS_CGS2)
  // column-blocked SpMV layout (when chosen): A by row panel and column block, its tiles
  int *col_pn = nullptr, *tiles_pn = nullptr, *toff_pn = nullptr, *ptile = nullptr;
  uint16_t* off_pn = nullptr;
  double* val_pn = nullptr;
  float* val32_pn = nullptr;
  double *Xr = nullptr, *ax1 = nullptr, *ax2 = nullptr, *rpart = nullptr;  // residual scratch (lazy)
  // E, B, S, cs and flags live in one device block and one pinned host block
  // of the same layout, so a restart moves them with one copy each way
  void* dstate = nullptr;
  void* hstate = nullptr;
  size_t bytes_pull = 0, bytes_push = 0;
  // pinned host mirrors
  double *hB = nullptr, *hS = nullptr, *hcs = nullptr, *hY = nullptr, *hE = nullptr;
  int* hflags = nullptr;
  // state
  int j = 0, q = 0, keff = 0, pending = 0;
  int keep = 0;  // restart size (kept Schur vectors), k <= keep <= m - 2
  int kr = 0;    // leading pairs tested and returned: k, or k + 1 to keep a conjugate pair
  int breakdowns = 0;  // replacement vectors drawn since the start (Philox counter of tag 3)
  int replaced = -1;   // last column replaced after a breakdown
  int64_t step_count = 0;  // Arnoldi steps run by this context (profiling sample clock)
  int G_z = 1, G_s = 1;
  bool have_state = false, solved = false;
  std::vector<double> Tk, bk;
  std::string err;
  // whole extensions recorded as HIP graphs, keyed by (start column, pending
  // column, basis precision): the launch sequence and every kernel argument
  // are fixed by that key, so the second occurrence of a key is recorded on a
  // private stream and every later one replays the graph on the solver's stream
  rks::LaunchEnv* lenv = nullptr;  // environment the step launchers use (env, or a copy while recording)
  hipStream_t cap = nullptr;
  std::map<int, hipGraphExec_t> gexec;
  std::map<int, int> gseen;
  std::map<int, std::pair<int, int>> gpart;  // G_z, G_s after the recorded extension
  // profiling
  std::vector<hipEvent_t> pool;
  std::vector<EvPair> open;
  size_t pool_used = 0;
  rks_stats* st = nullptr;
};

namespace {

// Failures of rks_create (no context exists yet) are reported per thread.
thread_local std::string g_create_err;

int fail(rks_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = std::string(code_str(code)) + ": " + msg;
  else
    g_create_err = std::string(code_str(code)) + ": " + msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail((ctx), RKS_EHIP, std::string(#call) + " -> " + hipGetErrorString(e_)); \
  } while (0)

void* basis_col(rks_ctx* c, int l) { return (char*)c->U + (size_t)l * c->ldu * c->vbytes; }

// ---- profiling -------------------------------------------------------------
enum { CAT_SPMV = 0, CAT_REDUCE, CAT_LS, CAT_UPDATE, CAT_ROTATE, CAT_STEP };

hipEvent_t get_event(rks_ctx* c) {
  if (c->pool_used == c->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->pool.push_back(e);
  }
  return c->pool[c->pool_used++];
}

struct Prof {
  rks_ctx* c;
  int cat;
  hipEvent_t a = nullptr;
  Prof(rks_ctx* c_, int cat_, bool on) : c(c_), cat(cat_) {
    if (on && c->o.profile > 0 && c->st) {
      a = get_event(c);
      if (a) (void)hipEventRecord(a, c->env.stream);
    }
  }
  ~Prof() {
    if (a) {
      hipEvent_t b = get_event(c);
      if (b) {
        (void)hipEventRecord(b, c->env.stream);
        c->open.push_back({cat, a, b});
      }
    }
  }
};

// Timing of one launcher's kernels from their own dispatch timestamps: the
// launcher gets a copy of the environment that carries two events (see
// LaunchEnv::ev0, ev1), so nothing is enqueued between the kernels.
struct ProfK {
  rks_ctx* c;
  int cat;
  rks::LaunchEnv env;
  ProfK(rks_ctx* c_, int cat_, bool on, const rks::LaunchEnv& e) : c(c_), cat(cat_), env(e) {
    env.ev0 = env.ev1 = nullptr;
    if (on && c->o.profile > 0 && c->st) {
      hipEvent_t a = get_event(c), b = a ? get_event(c) : nullptr;
      if (a && b) {
        env.ev0 = a;
        env.ev1 = b;
      }
    }
  }
  ~ProfK() {
    if (env.ev0) c->open.push_back({cat, env.ev0, env.ev1});
  }
};

void flush_events(rks_ctx* c) {
  if (!c->st) {
    c->open.clear();
    c->pool_used = 0;
    return;
  }
  for (auto& p : c->open) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) continue;
    double s = ms * 1e-3;
    switch (p.cat) {
      case CAT_SPMV: c->st->t_spmv += s; break;
      case CAT_STEP: c->st->t_step += s; break;
      case CAT_REDUCE: c->st->t_reduce += s; break;
      case CAT_LS: c->st->t_ls += s; break;
      case CAT_UPDATE: c->st->t_update += s; break;
      default: c->st->t_rotate += s; break;
    }
  }
  c->open.clear();
  c->pool_used = 0;
}

double spmv_bytes(const rks_ctx* c) {
  // A's values in FP64 for an FP64 or pair basis (whose SpMV reads the FP64 copy of its column),
  // or their one-byte indices (value-indexed storage)
  const bool f64 = c->env.prec == RKS_PREC_FP64 || c->pair;
  const double bval = f64 ? (c->env.vidx ? 1.0 : 8.0) : 4.0, xb = c->pair ? 8.0 : c->ebytes;
  return (bval + 4.0) * c->nnz + 4.0 * (c->n + 1) + (xb + c->wbytes) * c->n;
}

// The operand of the SpMV of column t: the column, or for the pair basis its FP64 copy.
const void* spmv_x(rks_ctx* c, int t) { return c->pair ? (const void*)c->xcur : basis_col(c, t); }
int spmv_prec(const rks_ctx* c) { return c->pair ? RKS_PREC_FP64 : -1; }

// ---- one Arnoldi step (Algorithm 2 loop body) ------------------------------
void account_step(rks_ctx* c, int t, bool timed, bool whole);

int arnoldi_step(rks_ctx* c, int t) {
  const auto& e = *c->lenv;
  // sampled timing: every P-th step, alternately per kernel and as a whole
  // (one event pair around the three launches, for the loop's bandwidth)
  bool timed = false, whole = false;
  if (c->o.profile > 0 && c->st && (c->step_count % c->o.profile) == 0) {
    if ((c->step_count / c->o.profile) % 2 == 0) timed = true;
    else whole = true;
  }
  ++c->step_count;
  Prof pw(c, CAT_STEP, whole);
  {
    ProfK p(c, CAT_SPMV, timed, e);
    c->G_z = rks::launch_spmv_sketch(p.env, spmv_x(c, t), c->w, c->zpart, 1, spmv_prec(c));
  }
  {
    ProfK p(c, CAT_REDUCE, timed, e);
    rks::launch_reduce(p.env, c->zpart, c->G_z, c->pending ? c->spart : nullptr, c->G_s, c->z, c->sr);
  }
  {
    // least squares and update in one launch (the least-squares time is
    // counted with the update)
    ProfK p(c, CAT_UPDATE, timed, e);
    c->G_s = rks::launch_ls_update(p.env, t, c->pending, c->z, c->sr, c->S, c->B, c->m + 1, c->E, c->cs, c->coef,
                                   c->scal, c->flags, kBreakdownRel, c->U, c->ldu, c->w, basis_col(c, t + 1),
                                   c->spart);
  }
  account_step(c, t, timed, whole);
  c->pending = 1;
  c->j = t + 1;
  return RKS_OK;
}

// Launch and byte counts of one randomized Arnoldi step.
void account_step(rks_ctx* c, int t, bool timed, bool whole) {
  if (!c->st) return;
  // the update reads t + 1 columns and w, writes one column (the pair basis:
  // and its FP64 copy)
  const double bs = spmv_bytes(c),
               bu = (double)(t + 2) * c->n * c->ebytes + (double)c->wbytes * c->n + (c->pair ? 8.0 * c->n : 0.0);
  c->st->n_spmv += 1;
  c->st->bytes_spmv += bs;
  c->st->n_update += 1;
  c->st->bytes_update += bu;
  c->st->matvecs += 1;
  if (timed) {
    c->st->n_timed_steps += 1;
    c->st->bytes_timed_spmv += bs;
    c->st->bytes_timed_update += bu;
  }
  if (whole) {
    c->st->n_timed_whole += 1;
    c->st->bytes_timed_whole += bs + bu;
  }
}

// ---- one Arnoldi step of deterministic Krylov-Schur ------------------------
// Classical Gram-Schmidt twice with the Euclidean inner product: two passes
// compute U^T x, two apply x - U y; the basis columns stay unnormalised with
// their scales in cs, as in the randomized step.
int arnoldi_step_ks(rks_ctx* c, int t) {
  const auto& e = c->env;
  bool timed = false, whole = false;
  if (c->o.profile > 0 && c->st && (c->step_count % c->o.profile) == 0) {
    if ((c->step_count / c->o.profile) % 2 == 0) timed = true;
    else whole = true;
  }
  ++c->step_count;
  Prof pw(c, CAT_STEP, whole);
  const int ncol = t + 1;
  void* unew = basis_col(c, t + 1);
  {
    Prof p(c, CAT_SPMV, timed);
    rks::launch_spmv_sketch(e, basis_col(c, t), c->w, nullptr, 0, -1);
  }
  {
    Prof p(c, CAT_UPDATE, timed);
    int G = rks::launch_dots(e, ncol, c->U, c->ldu, c->w, 0, c->kpart);
    rks::launch_reduce_len(e, c->kpart, G, c->z, ncol);
    rks::launch_ks_coef(e, ncol, c->cs, c->z, 1.0, c->cs + t, c->coef, c->sr, 0);
    rks::launch_update(e, ncol, c->U, c->ldu, c->w, c->coef, unew, c->spart);
    G = rks::launch_dots(e, ncol, c->U, c->ldu, unew, 1, c->kpart);
    rks::launch_reduce_len(e, c->kpart, G, c->z, ncol);
    rks::launch_ks_coef(e, ncol, c->cs, c->z, 1.0, nullptr, c->coef, c->sr, 1);
    const int Gs = rks::launch_update(e, ncol, c->U, c->ldu, unew, c->coef, unew, c->spart);
    rks::launch_reduce_len(e, c->spart, Gs, c->scal + 2, 1);
    rks::launch_ks_finalize(e, t, c->sr, c->scal + 2, c->B, c->m + 1, c->cs, c->flags, kBreakdownRel);
  }
  if (c->st) {
    const double bs = spmv_bytes(c), bu = (4.0 * (t + 1) + 6.0) * c->n * 8.0;
    c->st->n_spmv += 1;
    c->st->bytes_spmv += bs;
    c->st->n_update += 1;
    c->st->bytes_update += bu;
    c->st->matvecs += 1;
    if (timed) {
      c->st->n_timed_steps += 1;
      c->st->bytes_timed_spmv += bs;
      c->st->bytes_timed_update += bu;
    }
    if (whole) {
      c->st->n_timed_whole += 1;
      c->st->bytes_timed_whole += bs + bu;
    }
  }
  c->pending = 0;
  c->j = t + 1;
  return RKS_OK;
}

int finalize_last(rks_ctx* c) {
  const auto& e = *c->lenv;
  rks::launch_reduce(e, nullptr, 0, c->spart, c->G_s, c->z, c->sr);
  rks::launch_ls(e, c->j, 1, 1, c->z, c->sr, c->S, c->B, c->m + 1, c->E, c->cs, c->coef, c->scal, c->flags,
                 kBreakdownRel);
  c->pending = 0;
  return RKS_OK;
}

int extend_launch(rks_ctx* c) {
  for (int t = c->j; t < c->m; ++t) {
    int r = c->ks ? arnoldi_step_ks(c, t) : arnoldi_step(c, t);
    if (r) return r;
  }
  if (!c->ks) finalize_last(c);
  return RKS_OK;
}

int extend(rks_ctx* c) {
  const bool graphs = c->o.graphs && !c->ks && c->o.profile == 0 && c->j < c->m;
  const int key = (c->j * 2 + c->pending) * 4 + c->env.prec;
  if (graphs) {
    auto it = c->gexec.find(key);
    if (it != c->gexec.end()) {
      HIPCHK(c, hipGraphLaunch(it->second, c->env.stream));
      for (int t = c->j; t < c->m; ++t) account_step(c, t, false, false);
      c->j = c->m;
      c->pending = 0;
      c->G_z = c->gpart[key].first;
      c->G_s = c->gpart[key].second;
      return RKS_OK;
    }
    if (c->gseen[key]++ >= 1) {
      if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
      rks::LaunchEnv rec = c->env;
      rec.stream = c->cap;
      c->lenv = &rec;
      hipGraph_t g = nullptr;
      hipError_t e0 = hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed);
      const int rc = e0 == hipSuccess ? extend_launch(c) : RKS_OK;
      hipError_t e1 = e0 == hipSuccess ? hipStreamEndCapture(c->cap, &g) : e0;
      c->lenv = &c->env;
      if (rc) return rc;
      if (e1 != hipSuccess) return fail(c, RKS_EHIP, std::string("recording an extension -> ") + hipGetErrorString(e1));
      hipGraphExec_t ex = nullptr;
      hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) return fail(c, RKS_EHIP, std::string("hipGraphInstantiate -> ") + hipGetErrorString(e2));
      c->gexec[key] = ex;
      c->gpart[key] = {c->G_z, c->G_s};
      HIPCHK(c, hipGraphLaunch(ex, c->env.stream));
      return RKS_OK;
    }
  }
  const int rc = extend_launch(c);
  if (rc) return rc;
  HIPCHK(c, hipGetLastError());
  return RKS_OK;
}

int start(rks_ctx* c, const double* u0, int u0_on_device) {
  const double* u0d = nullptr;
  if (u0) {
    if (u0_on_device) {
      u0d = u0;
    } else {
      for (int64_t i = 0; i < c->n; ++i)
        if (!std::isfinite(u0[i])) return fail(c, RKS_ENAN, "u0 has a non-finite entry");
      HIPCHK(c, hipMemcpyAsync(c->u0tmp, u0, (size_t)c->n * 8, hipMemcpyHostToDevice, c->env.stream));
      u0d = c->u0tmp;
    }
  }
  const uint64_t s = c->o.start_seed;
  HIPCHK(c, hipMemsetAsync(c->B, 0, (size_t)(c->m + 1) * c->m * 8, c->env.stream));
  HIPCHK(c, hipMemsetAsync(c->S, 0, (size_t)c->d * (c->m + 1) * 8, c->env.stream));
  HIPCHK(c, hipMemsetAsync(c->flags, 0, sizeof(int) * 4, c->env.stream));
  HIPCHK(c, hipMemsetAsync(c->scal, 0, sizeof(double) * 4, c->env.stream));
  c->G_s = rks::launch_init(c->env, basis_col(c, 0), u0d, (uint32_t)s, (uint32_t)(s >> 32), c->spart, 1, -1);
  if (c->ks) {  // Euclidean normalisation of the start
    rks::launch_reduce_len(c->env, c->spart, c->G_s, c->scal + 2, 1);
    rks::launch_ks_start(c->env, c->scal + 2, c->cs);
  }
  HIPCHK(c, hipGetLastError());
  c->pending = c->ks ? 0 : 1;
  c->j = 0;
  c->q = 0;
  c->breakdowns = 0;
  c->replaced = -1;
  c->keff = 0;
  c->kr = 0;
  c->have_state = true;
  c->solved = false;
  return RKS_OK;
}

int pull_state(rks_ctx* c) {
  auto st = c->env.stream;
  // B, S, cs, flags: contiguous in both state blocks
  HIPCHK(c, hipMemcpyAsync(c->hB, c->B, c->bytes_pull, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  flush_events(c);
  return RKS_OK;
}

// Continuation past an exact invariant subspace (Section 2.1: the Krylov
// space has stopped growing, and the pairs it holds are exact).  The
// extension that found it (flags[0] = t: the remainder of A u_{t-1} vanished
// against its product) ran on to the end; its columns from t on are
// discarded.  Column t is replaced by a seeded N(0,1) vector (Philox tag 3,
// counter = number of replacements so far) sketch-orthogonalised against
// U_t by one least-squares and update launch; that launch also overwrites
// B(:, t-1) with the replacement's coefficients, so the pulled column is
// copied back, and flags[1] = t makes the finalisation of column t store
// B(t, t-1) = 0.  The extension then continues from column t.  It fails
// (RKS_EBREAKDOWN) only when the product with A of a replacement vector
// vanishes as well (flags[2]: the zero operator on that space).
int recover_breakdown(rks_ctx* c, int t) {
  const auto& e = c->env;
  const int ldb = c->m + 1;
  if (c->ks) return fail(c, RKS_EBREAKDOWN, "invariant subspace at column " + std::to_string(t));
  if (t < 1 || t > c->m || (c->hflags[2] != 0 && c->replaced == t - 1))
    return fail(c, RKS_EBREAKDOWN, "the product with A vanished for the replacement vector at column " +
                                       std::to_string(t - 1));
  c->breakdowns += 1;
  if (c->st) c->st->breakdowns += 1;
  const uint64_t s = c->o.start_seed;
  // w is FP64 (FP64 and pair bases), or FP32 with an FP32 or BF16 basis
  const int wprec = c->wbytes == 8 ? 0 : 1;
  const int G = rks::launch_init(e, c->w, nullptr, (uint32_t)s, (uint32_t)(s >> 32), c->zpart, 1, wprec,
                                 (uint32_t)c->breakdowns, 3u);
  rks::launch_reduce(e, c->zpart, G, nullptr, 0, c->z, nullptr);
  c->G_s = rks::launch_ls_update(e, t - 1, 0, c->z, c->sr, c->S, c->B, ldb, c->E, c->cs, c->coef, c->scal,
                                 c->flags, kBreakdownRel, c->U, c->ldu, c->w, basis_col(c, t), c->spart);
  HIPCHK(c, hipMemcpyAsync(c->B + (size_t)(t - 1) * ldb, c->hB + (size_t)(t - 1) * ldb, (size_t)t * 8,
                           hipMemcpyHostToDevice, e.stream));
  c->hflags[0] = 0;
  c->hflags[1] = t;
  c->hflags[2] = 0;
  HIPCHK(c, hipMemcpyAsync(c->flags, c->hflags, 3 * sizeof(int), hipMemcpyHostToDevice, e.stream));
  HIPCHK(c, hipGetLastError());
  c->replaced = t;
  c->j = t;
  c->pending = 1;
  return RKS_OK;
}

// Pull the state after an extension; while it reports a breakdown, replace
// the column and extend again (at most m times in a row).
int pull_and_recover(rks_ctx* c) {
  int rc = pull_state(c);
  for (int tries = 0; rc == RKS_OK && c->hflags[0] != 0; ++tries) {
    if (tries > c->m) return fail(c, RKS_EBREAKDOWN, "breakdown recovery did not end");
    rc = recover_breakdown(c, c->hflags[0]);
    if (rc == RKS_OK) rc = extend(c);
    if (rc == RKS_OK) rc = pull_state(c);
  }
  return rc;
}

// Ritz values/vectors of the truncated factor and the estimates.
// Only the leading kr x kr block (the wanted set) is used: T is quasi upper
// triangular, so its eigenvectors there have no components beyond kr.
void ritz(const rks_ctx* c, std::vector<cplx>& lam, std::vector<cplx>& Y, std::vector<double>& est) {
  const int kr = c->kr;
  lam.assign(kr, 0.0);
  Y.assign((size_t)kr * kr, 0.0);
  est.assign(kr, 0.0);
  rks::quasi_tri_eig(kr, c->Tk.data(), c->keff, lam.data(), Y.data());
  for (int i = 0; i < kr; ++i) {
    cplx s = 0.0;
    for (int r = 0; r < kr; ++r) s += c->bk[r] * Y[(size_t)r + (size_t)i * kr];
    est[i] = std::abs(s) / std::abs(lam[i]);
  }
}

// Dot product of two contiguous vectors with eight independent partial sums
// (a single running sum is one long dependent chain of FMAs).
double dot8(const double* a, const double* b, int n) {
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int r = 0;
  for (; r + 8 <= n; r += 8)
    for (int t = 0; t < 8; ++t) s[t] += a[r + t] * b[r + t];
  for (; r < n; ++r) s[r & 7] += a[r] * b[r];
  return ((s[0] + s[4]) + (s[1] + s[5])) + ((s[2] + s[6]) + (s[3] + s[7]));
}

// G = Sn^T Sn - I for the first nc columns of Sn (d rows), symmetric, into
// the (ld x ld) column-major array E.
void sketch_gram(const double* Sn, int d, int nc, double* E, int ld) {
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i <= j; ++i) {
      double g = dot8(&Sn[(size_t)i * d], &Sn[(size_t)j * d], d);
      if (i == j) g -= 1.0;
      E[i + (size_t)j * ld] = g;
      E[j + (size_t)i * ld] = g;
    }
}

// Contraction on the host: Schur form of the active block, reordering,
// truncation, whitening; fills Y for the device rotation and the new B, S,
// and E = S^T S - I of the contracted sketch (uploaded by push_state).
// Aggressive deflation (Section 4.4, after the deflation theorem: the
// decomposition may be reordered to test other Schur vectors for locking).
// Walks the nw wanted positions of the active Schur form (Ta, Z, ma x ma) in
// order; a block whose b entries (brow Z, brow with stride ldbr) pass the
// locking test of lock_converged once the block is moved to the front of the
// active part is moved there, so that the leading-block locking then takes
// it.  The other blocks keep their order behind the moved ones.
void front_converged(int ma, double* Ta, double* Z, const double* brow, int ldbr, int nw, double tol) {
  double tn = 0.0;
  for (int jj = 0; jj < nw; ++jj)
    for (int i = 0; i < nw; ++i) tn += Ta[i + (size_t)jj * ma] * Ta[i + (size_t)jj * ma];
  tn = std::sqrt(tn);
  std::vector<double> Tc((size_t)ma * ma), Zc((size_t)ma * ma);
  int pos = 0, idx = 0;
  while (idx < nw) {
    const int s = (idx + 1 < ma && Ta[(idx + 1) + (size_t)idx * ma] != 0.0) ? 2 : 1;
    const double* T1 = Ta;
    const double* Z1 = Z;
    if (idx != pos) {
      std::memcpy(Tc.data(), Ta, (size_t)ma * ma * 8);
      std::memcpy(Zc.data(), Z, (size_t)ma * ma * 8);
      if (rks::move_block(ma, Tc.data(), ma, Zc.data(), ma, idx, pos) != 0) {
        idx += s;
        continue;
      }
      T1 = Tc.data();
      Z1 = Zc.data();
    }
    const int sn = (pos + 1 < ma && T1[(pos + 1) + (size_t)pos * ma] != 0.0) ? 2 : 1;
    const double scale = std::max(std::abs(rks::block_eig(T1, ma, pos, sn)), kUnitRoundoff * tn);
    bool ok = true;
    for (int jj = pos; jj < pos + sn; ++jj) {
      double bv = 0.0;
      for (int l = 0; l < ma; ++l) bv += brow[(size_t)l * ldbr] * Z1[l + (size_t)jj * ma];
      ok = ok && std::fabs(bv) <= tol * scale;
    }
    if (ok) {
      if (idx != pos) {
        std::memcpy(Ta, Tc.data(), (size_t)ma * ma * 8);
        std::memcpy(Z, Zc.data(), (size_t)ma * ma * 8);
      }
      pos += sn;
    }
    idx += s;
  }
}

int contract(rks_ctx* c, int* in0, int* min, int* out0, int* kout, double* xscale, int* whitened) {
  const int m = c->m, q = c->q, k = c->k, d = c->d, ldb = m + 1;
  const int ma = m - q;
  double* hB = c->hB;
  std::vector<double> Ta((size_t)ma * ma), Z((size_t)ma * ma);
  for (int jj = 0; jj < ma; ++jj)
    for (int i = 0; i < ma; ++i) Ta[i + (size_t)jj * ma] = hB[(q + i) + (size_t)(q + jj) * ldb];
  for (double v : Ta)
    if (!std::isfinite(v)) return fail(c, RKS_ENAN, "non-finite Rayleigh quotient");
  if (rks::real_schur(ma, Ta.data(), ma, Z.data(), ma) != 0)
    return fail(c, RKS_EDENSE, "QR iteration did not converge");
  int p = 0;
  if (rks::order_wanted(ma, Ta.data(), ma, Z.data(), ma, c->which, c->keep - q, &p) != 0) {
    if (c->st) c->st->dense_fail += 1;
    if (p == 0) return fail(c, RKS_EDENSE, "reordering rejected every swap");
  }
  const int ke = q + p;
  c->keff = ke;
  // the wanted pairs: the leading k (the ordering is most wanted first), plus
  // one when a 2x2 block straddles column k
  int kr = std::min(k, ke);
  if (kr < ke && kr > q && Ta[(kr - q) + (size_t)(kr - 1 - q) * ma] != 0.0) kr += 1;
  c->kr = kr;
  if (c->o.lock == 2) front_converged(ma, Ta.data(), Z.data(), &hB[m + (size_t)q * ldb], ldb, kr - q, c->phase_tol);
  // truncated factor T (ke x ke) and b
  std::vector<double> T((size_t)ke * ke, 0.0), b(ke, 0.0);
  for (int jj = 0; jj < q; ++jj)
    for (int i = 0; i < q; ++i) T[i + (size_t)jj * ke] = hB[i + (size_t)jj * ldb];
  for (int jj = 0; jj < p; ++jj) {
    for (int i = 0; i < q; ++i) {
      double s = 0.0;
      for (int l = 0; l < ma; ++l) s += hB[i + (size_t)(q + l) * ldb] * Z[l + (size_t)jj * ma];
      T[i + (size_t)(q + jj) * ke] = s;
    }
    for (int i = 0; i < p; ++i) T[(q + i) + (size_t)(q + jj) * ke] = Ta[i + (size_t)jj * ma];
  }
  for (int i = 0; i < q; ++i) b[i] = hB[m + (size_t)i * ldb];
  for (int jj = 0; jj < p; ++jj) {
    double s = 0.0;
    for (int l = 0; l < ma; ++l) s += hB[m + (size_t)(q + l) * ldb] * Z[l + (size_t)jj * ma];
    b[q + jj] = s;
  }
  // truncated sketch S_new = S Q(:, 1:ke); last column is s_{m+1}
  std::vector<double> Sn((size_t)d * (ke + 1), 0.0);
  for (int i = 0; i < q; ++i) std::memcpy(&Sn[(size_t)i * d], &c->hS[(size_t)i * d], (size_t)d * 8);
  for (int jj = 0; jj < p; ++jj) {
    double* dst = &Sn[(size_t)(q + jj) * d];
    for (int l = 0; l < ma; ++l) {
      const double zv = Z[l + (size_t)jj * ma];
      if (zv == 0.0) continue;
      const double* src = &c->hS[(size_t)(q + l) * d];
      for (int r = 0; r < d; ++r) dst[r] += src[r] * zv;
    }
  }
  std::memcpy(&Sn[(size_t)ke * d], &c->hS[(size_t)m * d], (size_t)d * 8);
  // rotation matrix: Y = diag(cs) Q(:, 1:ke) (before whitening)
  std::vector<double> Yf((size_t)m * ke, 0.0);
  for (int i = 0; i < q; ++i) Yf[i + (size_t)i * m] = c->hcs[i];
  for (int jj = 0; jj < p; ++jj)
    for (int l = 0; l < ma; ++l) Yf[(q + l) + (size_t)(q + jj) * m] = c->hcs[q + l] * Z[l + (size_t)jj * ma];
  // whitening (Section 3.3) when the truncated sketch lost orthonormality
  const int ldE = m + 1;
  std::fill(c->hE, c->hE + (size_t)ldE * ldE, 0.0);
  if (!c->ks) sketch_gram(Sn.data(), d, ke + 1, c->hE, ldE);
  double dev = 0.0;
  for (int a = 0; a < ke; ++a)
    for (int bcol = 0; bcol < ke; ++bcol) dev += c->hE[a + (size_t)bcol * ldE] * c->hE[a + (size_t)bcol * ldE];
  dev = std::sqrt(dev);
  *whitened = 0;
  if (!c->ks && dev > c->o.whiten_tol) {  // deterministic Krylov-Schur keeps no sketch
    std::vector<double> Qs((size_t)d * ke), R((size_t)ke * ke), Ri((size_t)ke * ke);
    rks::householder_qr(d, ke, Sn.data(), d, Qs.data(), d, R.data(), ke);
    rks::upper_tri_inverse(ke, R.data(), ke, Ri.data(), ke);
    std::memcpy(Sn.data(), Qs.data(), (size_t)d * ke * 8);
    std::vector<double> T2((size_t)ke * ke, 0.0), T3((size_t)ke * ke, 0.0), b2(ke, 0.0), Y2((size_t)m * ke, 0.0);
    for (int jj = 0; jj < ke; ++jj)  // T2 = T Ri
      for (int l = 0; l <= jj; ++l) {
        const double rv = Ri[l + (size_t)jj * ke];
        for (int i = 0; i < ke; ++i) T2[i + (size_t)jj * ke] += T[i + (size_t)l * ke] * rv;
      }
    for (int jj = 0; jj < ke; ++jj)  // T3 = R T2
      for (int i = 0; i < ke; ++i) {
        double s = 0.0;
        for (int l = i; l < ke; ++l) s += R[i + (size_t)l * ke] * T2[l + (size_t)jj * ke];
        T3[i + (size_t)jj * ke] = s;
      }
    for (int jj = 0; jj < ke; ++jj) {
      double s = 0.0;
      for (int l = 0; l <= jj; ++l) s += b[l] * Ri[l + (size_t)jj * ke];
      b2[jj] = s;
    }
    for (int jj = 0; jj < ke; ++jj)
      for (int l = 0; l <= jj; ++l) {
        const double rv = Ri[l + (size_t)jj * ke];
        for (int i = 0; i < m; ++i) Y2[i + (size_t)jj * m] += Yf[i + (size_t)l * m] * rv;
      }
    T.swap(T3);
    b.swap(b2);
    Yf.swap(Y2);
    sketch_gram(Sn.data(), d, ke + 1, c->hE, ldE);
    *whitened = 1;
    if (c->st) c->st->whitenings += 1;
  }
  // choose the rotation extent: skip untouched locked columns
  bool lockedid = !*whitened;
  for (int i = 0; i < q && lockedid; ++i) lockedid = (c->hcs[i] == 1.0);
  if (lockedid) {
    *in0 = q; *min = m - q; *out0 = q; *kout = p;
    for (int jj = 0; jj < p; ++jj)
      for (int l = 0; l < ma; ++l) c->hY[l + (size_t)jj * ma] = Yf[(q + l) + (size_t)(q + jj) * m];
  } else {
    *in0 = 0; *min = m; *out0 = 0; *kout = ke;
    std::memcpy(c->hY, Yf.data(), (size_t)m * ke * 8);
  }
  *xscale = c->hcs[m];
  // new device-side state (uploaded by the caller after locking)
  std::fill(c->hB, c->hB + (size_t)(m + 1) * m, 0.0);
  for (int jj = 0; jj < ke; ++jj) {
    for (int i = 0; i < ke; ++i) hB[i + (size_t)jj * ldb] = T[i + (size_t)jj * ke];
    hB[ke + (size_t)jj * ldb] = b[jj];
  }
  std::fill(c->hS, c->hS + (size_t)d * (m + 1), 0.0);
  std::memcpy(c->hS, Sn.data(), (size_t)d * (ke + 1) * 8);
  for (int i = 0; i <= m; ++i) c->hcs[i] = 1.0;
  c->Tk = T;
  c->bk = b;
  return RKS_OK;
}

// Lock leading blocks of the wanted set whose b entries are small relative
// to their eigenvalue (Section 4.4, with the relative test) and zero them.
void lock_converged(rks_ctx* c) {
  const int ke = c->keff, ldb = c->m + 1;
  double tn = 0.0;
  for (double v : c->Tk) tn += v * v;
  tn = std::sqrt(tn);
  std::vector<int> st, sz;
  rks::blocks(ke, c->Tk.data(), ke, st, sz);
  int q = c->q;
  for (size_t bi = 0; bi < st.size(); ++bi) {
    if (st[bi] < q) continue;
    if (st[bi] != q || st[bi] + sz[bi] > c->kr) break;
    const double lam = std::abs(rks::block_eig(c->Tk.data(), ke, st[bi], sz[bi]));
    const double scale = std::max(lam, kUnitRoundoff * tn);
    bool ok = true;
    for (int i = st[bi]; i < st[bi] + sz[bi]; ++i) ok = ok && std::fabs(c->bk[i]) <= c->phase_tol * scale;
    if (!ok) break;
    q = st[bi] + sz[bi];
  }
  for (int i = 0; i < q; ++i) {
    c->bk[i] = 0.0;
    c->hB[ke + (size_t)i * ldb] = 0.0;
  }
  c->q = q;
}

int rotate_basis(rks_ctx* c, int in0, int min, int out0, int kout, double xscale) {
  auto stm = c->env.stream;
  HIPCHK(c, hipMemcpyAsync(c->Yd, c->hY, (size_t)min * kout * 8, hipMemcpyHostToDevice, stm));
  {
    ProfK p(c, CAT_ROTATE, true, c->env);
    rks::launch_rotate(p.env, c->U, c->ldu, in0, min, c->U, c->ldu, out0, kout, c->Yd, c->m, c->keff, xscale, 0);
  }
  HIPCHK(c, hipGetLastError());
  if (c->st) {
    const double br = (double)(min + 1 + kout + 1) * c->n * c->ebytes + (c->pair ? 8.0 * c->n : 0.0);
    c->st->n_rotate += 1;
    c->st->bytes_rotate += br;
    if (c->o.profile > 0) {
      c->st->n_timed_rotate += 1;
      c->st->bytes_timed_rotate += br;
    }
  }
  return RKS_OK;
}

int push_state(rks_ctx* c) {
  auto stm = c->env.stream;
  // E = S^T S - I of the contracted sketch (computed by contract), B, S and
  // cs: contiguous in both state blocks
  HIPCHK(c, hipMemcpyAsync(c->E, c->hE, c->bytes_push, hipMemcpyHostToDevice, stm));
  c->j = c->keff;
  c->pending = 0;
  return RKS_OK;
}

// Ritz pairs sorted by `which` and the real packing matrix W (ke x ke) with
// x = U_k W: a conjugate pair occupies two columns (real, imaginary part).
struct Packed {
  std::vector<cplx> lam;
  std::vector<double> W;
  std::vector<int> pair_of;  // 0 real, 1 first of a pair, 2 second
};

Packed pack_ritz(const rks_ctx* c) {
  const int ke = c->kr;
  std::vector<cplx> lam, Y;
  std::vector<double> est;
  ritz(c, lam, Y, est);
  std::vector<int> ord(ke);
  for (int i = 0; i < ke; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return rks::more_wanted(lam[a], lam[b], c->which); });
  Packed P;
  P.lam.resize(ke);
  P.W.assign((size_t)ke * ke, 0.0);
  P.pair_of.assign(ke, 0);
  for (int i = 0; i < ke; ++i) P.lam[i] = lam[ord[i]];
  for (int i = 0; i < ke;) {
    const cplx* y = &Y[(size_t)ord[i] * ke];
    if (P.lam[i].imag() != 0.0 && i + 1 < ke) {
      for (int r = 0; r < ke; ++r) {
        P.W[r + (size_t)i * ke] = y[r].real();
        P.W[r + (size_t)(i + 1) * ke] = y[r].imag();
      }
      P.pair_of[i] = 1;
      P.pair_of[i + 1] = 2;
      i += 2;
    } else {
      for (int r = 0; r < ke; ++r) P.W[r + (size_t)i * ke] = y[r].real();
      i += 1;
    }
  }
  return P;
}

int ensure_resid_scratch(rks_ctx* c) {
  const size_t cols = (size_t)c->k + 1;
  if (!c->Xr && hipMalloc(&c->Xr, (size_t)c->n * cols * 8) != hipSuccess) return fail(c, RKS_ENOMEM, "residual X");
  if (!c->ax1 && hipMalloc(&c->ax1, (size_t)c->n * 8) != hipSuccess) return fail(c, RKS_ENOMEM, "residual AX");
  if (!c->ax2 && hipMalloc(&c->ax2, (size_t)c->n * 8) != hipSuccess) return fail(c, RKS_ENOMEM, "residual AX");
  if (!c->rpart && hipMalloc(&c->rpart, cols * 2 * rks::kMaxG * 8) != hipSuccess)
    return fail(c, RKS_ENOMEM, "residual partials");
  return RKS_OK;
}

// X = U_k W on the device (FP64, n x ke, leading dimension n), then the FP64
// residual of every pair; optionally X columns are normalised to unit norm.
int device_residuals(rks_ctx* c, const Packed& P, double* Xd, double* resid, bool normalise) {
  auto stm = c->env.stream;
  const int ke = c->kr;
  const int64_t n = c->n;
  HIPCHK(c, hipStreamSynchronize(stm));  // the pinned staging buffer hY may still be in flight
  for (int c0 = 0; c0 < ke; c0 += rks::kRotMax) {
    const int kc = std::min(rks::kRotMax, ke - c0);
    for (int jj = 0; jj < kc; ++jj)
      for (int r = 0; r < ke; ++r) c->hY[r + (size_t)jj * ke] = P.W[r + (size_t)(c0 + jj) * ke];
    HIPCHK(c, hipMemcpyAsync(c->Yd, c->hY, (size_t)ke * kc * 8, hipMemcpyHostToDevice, stm));
    rks::launch_rotate(c->env, c->U, c->ldu, 0, ke, Xd, n, c0, kc, c->Yd, -1, 0, 0.0, 1);
    HIPCHK(c, hipStreamSynchronize(stm));  // hY is reused by the next chunk
  }
  // every pair's products and partial sums first (slot s of rpart, stride
  // 2 G), then one copy and one synchronisation for all of them; the AX
  // buffers are reused in stream order
  std::vector<int> first;
  int G = 0;
  for (int i = 0; i < ke;) {
    const bool cp = P.pair_of[i] == 1;
    double* xa = Xd + (size_t)i * n;
    double* xb = cp ? Xd + (size_t)(i + 1) * n : nullptr;
    rks::launch_spmv_sketch(c->env, xa, c->ax1, nullptr, 0, 0);
    if (cp) rks::launch_spmv_sketch(c->env, xb, c->ax2, nullptr, 0, 0);
    G = rks::launch_resid(c->env, xa, xb, c->ax1, cp ? c->ax2 : nullptr, P.lam[i].real(), P.lam[i].imag(),
                          c->rpart + first.size() * 2 * rks::kMaxG);
    first.push_back(i);
    i += cp ? 2 : 1;
  }
  HIPCHK(c, hipGetLastError());
  std::vector<double> hpart(first.size() * 2 * rks::kMaxG);
  HIPCHK(c, hipMemcpyAsync(hpart.data(), c->rpart, hpart.size() * 8, hipMemcpyDeviceToHost, stm));
  HIPCHK(c, hipStreamSynchronize(stm));
  for (size_t sl = 0; sl < first.size(); ++sl) {
    const int i = first[sl];
    const bool cp = P.pair_of[i] == 1;
    const double* hp = &hpart[sl * 2 * rks::kMaxG];
    double rr = 0.0, xx = 0.0;
    for (int g = 0; g < G; ++g) {
      rr += hp[2 * g];
      xx += hp[2 * g + 1];
    }
    const double res = std::sqrt(rr) / (c->normA1 * std::sqrt(xx));
    if (normalise) {
      const double sc = 1.0 / std::sqrt(xx);
      rks::launch_scale(c->env, Xd + (size_t)i * n, sc);
      if (cp) rks::launch_scale(c->env, Xd + (size_t)(i + 1) * n, sc);
    }
    resid[i] = res;
    if (cp) resid[i + 1] = res;
  }
  HIPCHK(c, hipGetLastError());
  return RKS_OK;
}

// Largest FP64 residual of the current wanted pairs, verified on the device.
int verified_max_resid(rks_ctx* c, double* out) {
  int rc = ensure_resid_scratch(c);
  if (rc) return rc;
  Packed P = pack_ritz(c);
  std::vector<double> res(c->kr, 0.0);
  rc = device_residuals(c, P, c->Xr, res.data(), false);
  if (rc) return rc;
  double mr = 0.0;
  for (double v : res) mr = std::max(mr, v);
  *out = mr;
  return RKS_OK;
}

// Switch the basis in use between the requested precision and FP64.
int set_basis(rks_ctx* c, int prec) {
  c->env.prec = prec;
  c->pair = prec == RKS_PREC_V32_FX16;
  c->vbytes = (prec == RKS_PREC_FP64) ? 8 : (prec == RKS_PREC_VBF16 ? 2 : 4);
  c->ebytes = c->pair ? 6 : c->vbytes;
  c->wbytes = (prec == RKS_PREC_FP64 || c->pair) ? 8 : 4;
  if (prec == c->o.precision) {
    c->U = c->U_lo;
  } else {
    if (!c->U64) {
      const size_t bytes = (size_t)c->ldu * (c->m + 1) * 8;
      if (hipMalloc(&c->U64, bytes) != hipSuccess) {
        c->U64 = nullptr;
        return fail(c, RKS_ENOMEM, "FP64 refinement basis");
      }
      HIPCHK(c, hipMemsetAsync(c->U64, 0, bytes, c->env.stream));
    }
    c->U = c->U64;
  }
  return RKS_OK;
}

struct PhaseOut {
  int restarts;
  int reason;
  int resid_checks;
  double maxest, maxres, thost;
};

// Algorithm 1 from u0 until the estimates reach tol, the verified residual
// reaches resid_tol (> 0), or max_restarts cycles.
int run_phase(rks_ctx* c, const double* u0, int u0_on_device, double tol, double resid_tol, int max_restarts,
              int hist_off, PhaseOut* out) {
  rks_stats* st = c->st;
  c->phase_tol = tol;
  *out = PhaseOut{0, 0, 0, 0.0, 0.0, 0.0};
  int rc = start(c, u0, u0_on_device);
  if (rc) return rc;
  rc = extend(c);
  if (rc) return rc;
  int restarts = 0, reason = 0;
  double maxest = 0.0, maxres = 0.0, last_fail_pred = INFINITY, thost = 0.0;
  // stagnation: the restart at which the largest estimate last halved
  double stall_mark = INFINITY;
  int stall_at = 0;
  // true max residual / predicted max residual at the last failed verification
  // (the predicted residual |b^T y| / ||A||_1 misses the embedding's distortion
  // of ||u_{k+1}|| / ||x||, so the two differ by a slowly varying factor)
  double ratio = 1.0;
  while (true) {
    rc = pull_and_recover(c);
    if (rc) break;
    const auto h0 = std::chrono::steady_clock::now();
    int in0, min, out0, kout, wh;
    double xscale;
    rc = contract(c, &in0, &min, &out0, &kout, &xscale, &wh);
    if (rc) break;
    std::vector<cplx> lam, Y;
    std::vector<double> est;
    ritz(c, lam, Y, est);
    maxest = 0.0;
    double pred = 0.0;  // estimated backward residual relative to ||A||_1
    bool allfinite = true;
    for (int i = 0; i < (int)est.size(); ++i) {
      if (!std::isfinite(est[i])) allfinite = false;
      maxest = std::max(maxest, est[i]);
      pred = std::max(pred, est[i] * std::abs(lam[i]) / c->normA1);
    }
    if (!allfinite) maxest = pred = INFINITY;
    if (hist_off + restarts < 512) st->hist_est[hist_off + restarts] = maxest;
    const bool converged = allfinite && maxest <= tol;
    thost += std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
    rc = rotate_basis(c, in0, min, out0, kout, xscale);
    if (rc) break;
    if (converged) {
      reason = 1;
    } else if (resid_tol > 0.0 && allfinite && pred <= resid_tol && pred <= 0.9 * last_fail_pred &&
               (pred * ratio <= resid_tol || pred <= 0.5 * last_fail_pred)) {
      // the estimates predict the target residual: verify it in FP64 on the device
      rc = ensure_resid_scratch(c);
      if (rc) break;
      Packed P = pack_ritz(c);
      std::vector<double> res(c->kr, 0.0);
      rc = device_residuals(c, P, c->Xr, res.data(), false);
      if (rc) break;
      out->resid_checks += 1;
      double mr = 0.0;
      for (double v : res) mr = std::max(mr, v);
      if (mr <= resid_tol) {
        reason = 2;
        maxres = mr;
      } else {
        last_fail_pred = pred;
        ratio = std::max(mr / std::max(pred, 1e-300), 1e-3);
      }
    }
    if (reason == 0 && allfinite) {
      if (maxest < 0.5 * stall_mark) {
        stall_mark = maxest;
        stall_at = restarts;
      } else if (c->o.stall_restarts > 0 && restarts - stall_at >= c->o.stall_restarts) {
        reason = 3;
      }
    }
    const bool stop = reason != 0 || restarts >= max_restarts;
    if (!stop && c->o.lock) lock_converged(c);
    rc = push_state(c);
    if (rc) break;
    if (stop) break;
    rc = extend(c);
    if (rc) break;
    ++restarts;
  }
  out->restarts = restarts;
  out->reason = reason;
  out->maxest = maxest;
  out->maxres = maxres;
  out->thost = thost;
  return rc;
}

// Start vector of the FP64 phase: a fixed combination of the low-precision
// Schur vectors U_k (which span the approximate wanted invariant subspace),
// formed in FP64 on the device into u0tmp; then switch the basis to FP64.
int refine_start(rks_ctx* c) {
  const int ke = c->kr;
  HIPCHK(c, hipStreamSynchronize(c->env.stream));
  for (int i = 0; i < ke; ++i) c->hY[i] = 1.0 + 0.25 * (i % 3);
  HIPCHK(c, hipMemcpyAsync(c->Yd, c->hY, (size_t)ke * 8, hipMemcpyHostToDevice, c->env.stream));
  rks::launch_rotate(c->env, c->U, c->ldu, 0, ke, c->u0tmp, c->n, 0, 1, c->Yd, -1, 0, 0.0, 1);
  HIPCHK(c, hipGetLastError());
  return set_basis(c, RKS_PREC_FP64);
}

bool valid_csr(const int32_t* rp, const int32_t* col, int64_t n, int64_t nnz, std::string& why) {
  if (rp[0] != 0) { why = "row_ptr[0] != 0"; return false; }
  if (rp[n] != nnz) { why = "row_ptr[n] != nnz"; return false; }
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) { why = "row_ptr not monotone"; return false; }
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) { why = "column index out of range"; return false; }
      if (e > rp[i] && col[e] <= col[e - 1]) { why = "columns not strictly increasing in a row"; return false; }
    }
  }
  return true;
}

void free_all(rks_ctx* c) {
  void* dev[] = {c->rp, c->col, c->tiles, c->dstate, c->val, c->val32, c->U_lo, c->U64, c->w, c->xcur,
                 c->coef, c->z, c->sr, c->zpart, c->spart, c->scal, c->Yd, c->u0tmp, c->kpart,
                 c->col_pn, c->tiles_pn, c->toff_pn, c->ptile, c->off_pn, c->val_pn, c->val32_pn,
                 c->Xr, c->ax1, c->ax2, c->rpart, c->vidx, c->vtab, c->sl_off, c->col_sl, c->val_sl,
                 c->vidx_sl, c->val32_sl};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {c->hstate, c->hY};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  for (auto e : c->pool) (void)hipEventDestroy(e);
  for (auto& kv : c->gexec) (void)hipGraphExecDestroy(kv.second);
  if (c->cap) (void)hipStreamDestroy(c->cap);
}

}  // namespace

extern "C" {

void rks_opts_default(rks_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sketch_kind = RKS_SKETCH_SPARSE;
  o->zeta = 8;
  o->sketch_seed = 0;
  o->start_seed = 1;
  o->precision = RKS_PREC_FP64;
  o->max_restarts = 300;
  o->lock = 1;
  o->profile = 0;
  o->whiten_tol = 1e-12;
  o->stream = nullptr;
  o->resid_tol = 0.0;
  o->refine = 1;
  o->refine_tol = 0.0;
  o->spmv_layout = RKS_SPMV_AUTO;
  o->method = RKS_METHOD_RKS;
  o->keep = 0;
  o->graphs = 0;
}

const char* rks_strerror(int code) { return code_str(code); }

const char* rks_last_error(const rks_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int rks_create(const rks_csr* A, int32_t k, int32_t m, int32_t d, int32_t which, double tol, const rks_opts* opts,
               rks_ctx** out) {
  g_create_err.clear();
  if (!out) return fail(nullptr, RKS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!A || !A->row_ptr || (A->nnz > 0 && (!A->col || !A->val))) return fail(nullptr, RKS_EINVAL, "CSR pointers");
  const int64_t n = A->n, nnz = A->nnz;
  rks_opts o;
  if (opts) o = *opts; else rks_opts_default(&o);
  if (n < 4 || nnz < 0 || nnz >= (int64_t)1 << 31 || n >= (int64_t)1 << 31)
    return fail(nullptr, RKS_EINVAL, "need 4 <= n < 2^31 and nnz < 2^31");
  if (k < 1 || k + 2 > m || m > rks::kMaxM || m + 1 > d || d > n || d > rks::kMaxD)
    return fail(nullptr, RKS_EINVAL, "need 1 <= k, k+2 <= m <= 255, m+1 <= d <= min(n, 1024)");
  if (k + 1 > rks::kRotMax) return fail(nullptr, RKS_EINVAL, "need k + 1 <= 128");
  if (!(tol > 0.0) || which < 0 || which > 3) return fail(nullptr, RKS_EINVAL, "tol or which");
  if (o.sketch_kind != RKS_SKETCH_GAUSS && o.sketch_kind != RKS_SKETCH_SPARSE)
    return fail(nullptr, RKS_EINVAL, "sketch_kind");
  if (o.sketch_kind == RKS_SKETCH_SPARSE && (o.zeta < 1 || o.zeta > 8 || o.zeta > d))
    return fail(nullptr, RKS_EINVAL, "need 1 <= zeta <= min(8, d)");
  if (o.precision < 0 || o.precision > 3 || o.max_restarts < 0 || !(o.whiten_tol >= 0.0) ||
      !(o.resid_tol >= 0.0) || !(o.refine_tol >= 0.0) || o.spmv_layout < 0 || o.spmv_layout > 3 || o.method < 0 ||
      o.method > 1 || o.graphs < 0 || o.graphs > 1 || o.stall_restarts < 0 || o.a_values < 0 || o.a_values > 1)
    return fail(nullptr, RKS_EINVAL,
                "precision, max_restarts, whiten_tol, resid_tol, refine_tol, spmv_layout, method, graphs, "
                "stall_restarts or a_values");
  int keep = o.keep == 0 ? k : o.keep;
  if (o.keep == RKS_KEEP_AUTO)
    keep = std::max(k, std::min({k + (m - k) / 4, m - 2, rks::kRotMax - 1}));
  if (keep < k || keep + 2 > m || keep + 1 > rks::kRotMax)
    return fail(nullptr, RKS_EINVAL, "need k <= keep <= m - 2 and keep + 1 <= 128");
  if (o.method == RKS_METHOD_KS_CGS2 && o.precision != RKS_PREC_FP64)
    return fail(nullptr, RKS_EINVAL, "deterministic Krylov-Schur runs with an FP64 basis only");
  if (o.lock < 0 || o.lock > 2) return fail(nullptr, RKS_EINVAL, "lock must be 0, 1 or 2");

  rks_ctx* c = new (std::nothrow) rks_ctx();
  if (!c) return fail(nullptr, RKS_ENOMEM, "context");
  c->n = n; c->nnz = nnz; c->k = k; c->m = m; c->d = d; c->which = which; c->tol = tol; c->o = o;
  c->lenv = &c->env;
  c->keep = keep;
  hipStream_t stm = (hipStream_t)o.stream;
  // host copies for validation, the 1-norm and the SpMV tiles
  std::vector<int32_t> rp(n + 1), col(nnz);
  std::vector<double> val(nnz);
  if (A->on_device) {
    if (hipMemcpy(rp.data(), A->row_ptr, (n + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        (nnz && hipMemcpy(col.data(), A->col, nnz * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
        (nnz && hipMemcpy(val.data(), A->val, nnz * 8, hipMemcpyDeviceToHost) != hipSuccess)) {
      delete c;
      return fail(nullptr, RKS_EHIP, "copying the device CSR to the host");
    }
  } else {
    std::memcpy(rp.data(), A->row_ptr, (n + 1) * 4);
    if (nnz) {
      std::memcpy(col.data(), A->col, nnz * 4);
      std::memcpy(val.data(), A->val, nnz * 8);
    }
  }
  std::string why;
  if (!valid_csr(rp.data(), col.data(), n, nnz, why)) {
    delete c;
    return fail(nullptr, RKS_EINVAL, why);
  }
  std::vector<double> colsum(n, 0.0);
  for (int64_t e = 0; e < nnz; ++e) {
    if (!std::isfinite(val[e])) {
      delete c;
      return fail(nullptr, RKS_ENAN, "non-finite value in A");
    }
    colsum[col[e]] += std::fabs(val[e]);
  }
  c->normA1 = n ? *std::max_element(colsum.begin(), colsum.end()) : 0.0;
  // wave tiles: <= 64 rows and <= 512 nonzeros, or one long row;
  // descriptors {first row, rows, first nonzero, nonzeros} appended to out
  auto build_tiles = [&](const int32_t* rpx, std::vector<int32_t>& out) {
    for (int64_t r = 0; r < n;) {
      const int64_t s0 = r;
      int64_t acc = 0;
      if (rpx[r + 1] - rpx[r] > rks::kTileFill) {
        ++r;
      } else {
        while (r < n && r - s0 < rks::kTileRows && acc + (rpx[r + 1] - rpx[r]) <= rks::kTileFill) {
          acc += rpx[r + 1] - rpx[r];
          ++r;
        }
      }
      out.push_back((int32_t)s0);
      out.push_back((int32_t)(r - s0));
      out.push_back(rpx[s0]);
      out.push_back(rpx[r] - rpx[s0]);
    }
  };
  std::vector<int32_t> tdesc;
  build_tiles(rp.data(), tdesc);
  const int ntiles = (int)(tdesc.size() / 4);
  // column-blocked layout for operators whose rows gather x from everywhere
  bool use_cb = o.spmv_layout == RKS_SPMV_COLUMN_BLOCKS;
  if (o.spmv_layout == RKS_SPMV_AUTO && n >= (1 << 20)) {
    std::vector<int64_t> spans;
    const int step = std::max(1, ntiles / 4096);
    for (int t = 0; t < ntiles; t += step) {
      const int64_t e0 = tdesc[4 * t + 2], ne = tdesc[4 * t + 3];
      if (ne == 0) continue;
      int32_t lo = col[e0], hi = col[e0];
      for (int64_t e = e0; e < e0 + ne; ++e) {
        lo = std::min(lo, col[e]);
        hi = std::max(hi, col[e]);
      }
      spans.push_back(hi - lo);
    }
    if (!spans.empty()) {
      std::nth_element(spans.begin(), spans.begin() + spans.size() / 2, spans.end());
      use_cb = spans[spans.size() / 2] > n / 4;
    }
  }
  rks::PanelLayout pl;
  if (use_cb && !rks::build_panels(n, rp.data(), col.data(), val.data(), pl, why)) {
    delete c;
    return fail(nullptr, RKS_EINVAL, why);
  }
  const bool pair = o.precision == RKS_PREC_V32_FX16;
  const bool low = o.precision == RKS_PREC_V32 || o.precision == RKS_PREC_VBF16;  // FP32 copies of A's values
  // value-indexed storage for the FP64 product (row tiles): the table of
  // distinct values (bit patterns, at most 256, kept sorted) and each
  // nonzero's index into it
  std::vector<uint64_t> vkeys;
  std::vector<uint8_t> vind;
  int a_nd = 0;  // distinct values of A (the table may hold +0.0 besides)
  if (o.a_values == RKS_AVALUES_AUTO && !use_cb && nnz > 0) {
    for (int64_t e = 0; e < nnz && vkeys.size() <= 256; ++e) {
      uint64_t key;
      std::memcpy(&key, &val[e], 8);
      auto it = std::lower_bound(vkeys.begin(), vkeys.end(), key);
      if (it == vkeys.end() || *it != key) vkeys.insert(it, key);
    }
    if (vkeys.size() <= 256) {
      a_nd = (int)vkeys.size();
      // +0.0 in the table (if there is room) pads the sliced layout
      if (vkeys.front() != 0 && vkeys.size() < 256) vkeys.insert(vkeys.begin(), (uint64_t)0);
      vind.resize(nnz);
      for (int64_t e = 0; e < nnz; ++e) {
        uint64_t key;
        std::memcpy(&key, &val[e], 8);
        vind[e] = (uint8_t)(std::lower_bound(vkeys.begin(), vkeys.end(), key) - vkeys.begin());
      }
    } else {
      vkeys.clear();
    }
  }
  const bool indexed = !vkeys.empty();
  // sliced layout: slices of kSliceRows rows, each padded to its longest row
  const int64_t nsl = (n + rks::kSliceRows - 1) / rks::kSliceRows;
  std::vector<int64_t> sloff;
  bool use_sl = false;
  if (!use_cb && (o.spmv_layout == RKS_SPMV_SLICED || o.spmv_layout == RKS_SPMV_AUTO)) {
    rks::slice_offsets(n, rp.data(), sloff);
    const int64_t P = sloff[nsl];
    use_sl = (o.spmv_layout == RKS_SPMV_SLICED || P <= nnz + nnz / 8) && P > 0 && P < ((int64_t)1 << 31);
    if (o.spmv_layout == RKS_SPMV_SLICED && !use_sl) {
      delete c;
      return fail(nullptr, RKS_EINVAL, "sliced layout: no nonzeros, or 2^31 padded entries or more");
    }
  }
  const int64_t sl_entries = use_sl ? sloff[nsl] : 0;
  // padding carries the value +0.0, so the kernel may add it (no row lengths
  // needed), unless the value table is full without +0.0
  const bool pad0 = !indexed || vkeys.front() == 0;
  const int ebytes = o.precision == RKS_PREC_FP64 ? 8 : (pair ? 6 : (o.precision == RKS_PREC_V32 ? 4 : 2));
  c->ldu = (n + 127) / 128 * 128;
  c->pair = pair;
  c->vbytes = o.precision == RKS_PREC_FP64 ? 8 : (o.precision == RKS_PREC_VBF16 ? 2 : 4);
  c->ebytes = ebytes;
  c->wbytes = (o.precision == RKS_PREC_FP64 || pair) ? 8 : 4;
  bool ok = true;
  std::string what;
  auto dm = [&](void** p, size_t bytes) {
    if (!ok) return;
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) {
      ok = false;
      what = "hipMalloc(" + std::to_string(bytes) + ") -> " + hipGetErrorString(e);
    }
  };
  auto hm = [&](void** p, size_t bytes) {
    if (!ok) return;
    hipError_t e = hipHostMalloc(p, bytes ? bytes : 8, hipHostMallocDefault);
    if (e != hipSuccess) {
      ok = false;
      what = "hipHostMalloc(" + std::to_string(bytes) + ") -> " + hipGetErrorString(e);
    }
  };
  dm((void**)&c->rp, (n + 1) * 4);
  const int64_t nzp = nnz + rks::kCsrPad;  // padded: the SpMV reads nonzeros in aligned pairs
  dm((void**)&c->col, nzp * 4);
  dm((void**)&c->val, nzp * 8);
  if (low) dm((void**)&c->val32, nzp * 4);
  if (indexed) {
    dm((void**)&c->vidx, nzp);
    dm((void**)&c->vtab, 256 * 8);
  }
  if (use_sl) {
    dm((void**)&c->sl_off, (size_t)(nsl + 1) * 8);
    dm((void**)&c->col_sl, (size_t)sl_entries * 4);
    if (indexed) dm((void**)&c->vidx_sl, (size_t)sl_entries);
    else dm((void**)&c->val_sl, (size_t)sl_entries * 8);
    if (low) dm((void**)&c->val32_sl, (size_t)sl_entries * 4);
  }
  dm((void**)&c->tiles, tdesc.size() * 4);
  if (use_cb) {
    dm((void**)&c->col_pn, (size_t)nzp * 4);
    dm((void**)&c->val_pn, (size_t)nzp * 8);
    if (low) dm((void**)&c->val32_pn, (size_t)nzp * 4);
    dm((void**)&c->tiles_pn, pl.tiles.size() * 4);
    dm((void**)&c->toff_pn, pl.toff.size() * 4);
    dm((void**)&c->off_pn, pl.off.size() * 2);
    dm((void**)&c->ptile, pl.ptile.size() * 4);
  }
  dm(&c->U_lo, (size_t)c->ldu * (m + 1) * ebytes);
  c->U = c->U_lo;
  dm(&c->w, (size_t)c->ldu * 8);
  if (pair) dm((void**)&c->xcur, (size_t)c->ldu * 8);
  // state block: E ((m+1)^2) | B ((m+1) m) | S (d (m+1)) | cs (m+1) | flags (4 int32), FP64 offsets
  const size_t oE = 0, oB = oE + (size_t)(m + 1) * (m + 1), oS = oB + (size_t)(m + 1) * m,
               oC = oS + (size_t)d * (m + 1), oF = oC + (size_t)(m + 1), state_bytes = (oF + 2) * 8;
  dm(&c->dstate, state_bytes);
  hm(&c->hstate, state_bytes);
  if (ok) {
    double* ds = (double*)c->dstate;
    double* hs = (double*)c->hstate;
    c->E = ds + oE; c->B = ds + oB; c->S = ds + oS; c->cs = ds + oC; c->flags = (int*)(ds + oF);
    c->hE = hs + oE; c->hB = hs + oB; c->hS = hs + oS; c->hcs = hs + oC; c->hflags = (int*)(hs + oF);
    c->bytes_pull = (oF + 2 - oB) * 8;
    c->bytes_push = (oF - oE) * 8;
  }
  dm((void**)&c->coef, (size_t)(m + 2) * 8);
  dm((void**)&c->z, (size_t)d * 8);
  dm((void**)&c->sr, (size_t)d * 8);
  dm((void**)&c->zpart, (size_t)std::max<int64_t>(rks::kMaxPart, pl.npanels) * d * 8);
  dm((void**)&c->spart, (size_t)rks::kMaxG * d * 8);
  dm((void**)&c->scal, 8 * 8);
  dm((void**)&c->Yd, (size_t)(m + 1) * (m + 1) * 8);
  dm((void**)&c->u0tmp, (size_t)n * 8);
  if (o.method == RKS_METHOD_KS_CGS2) dm((void**)&c->kpart, (size_t)rks::kMaxG * (m + 1) * 8);
  hm((void**)&c->hY, (size_t)(m + 1) * (m + 1) * 8);
  if (!ok) {
    free_all(c);
    delete c;
    return fail(nullptr, RKS_ENOMEM, what);
  }
  int rc = RKS_OK;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (rc == RKS_OK && bytes && hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) rc = RKS_EHIP;
  };
  cp(c->rp, rp.data(), (n + 1) * 4);
  cp(c->col, col.data(), nnz * 4);
  cp(c->val, val.data(), nnz * 8);
  if (c->val32) {
    std::vector<float> v32(val.begin(), val.end());
    cp(c->val32, v32.data(), nnz * 4);
  }
  if (indexed) {
    std::vector<double> tab(256, 0.0);
    for (size_t i = 0; i < vkeys.size(); ++i) std::memcpy(&tab[i], &vkeys[i], 8);
    cp(c->vidx, vind.data(), nnz);
    cp(c->vtab, tab.data(), 256 * 8);
    c->a_distinct = a_nd;
  }
  if (use_sl && rc == RKS_OK) {
    // columns of the entries, and their values: padding carries +0.0 (table
    // index 0 when value-indexed and pad0), so it adds exactly 0 for finite x
    std::vector<int32_t> scol, src;
    rks::build_slices(n, rp.data(), col.data(), sloff, scol, src);
    std::vector<uint8_t> sidx(indexed ? (size_t)sl_entries : 0);
    std::vector<double> sval(indexed ? 0 : (size_t)sl_entries);
    std::vector<float> sval32(low ? (size_t)sl_entries : 0);
    for (size_t e = 0; e < (size_t)sl_entries; ++e) {
      const int32_t j = src[e];
      if (indexed) sidx[e] = j >= 0 ? vind[j] : 0;
      else sval[e] = j >= 0 ? val[j] : 0.0;
      if (low) sval32[e] = j >= 0 ? (float)val[j] : 0.0f;
    }
    cp(c->sl_off, sloff.data(), (size_t)(nsl + 1) * 8);
    cp(c->col_sl, scol.data(), (size_t)sl_entries * 4);
    if (indexed) cp(c->vidx_sl, sidx.data(), (size_t)sl_entries);
    else cp(c->val_sl, sval.data(), (size_t)sl_entries * 8);
    if (low) cp(c->val32_sl, sval32.data(), (size_t)sl_entries * 4);
  }
  cp(c->tiles, tdesc.data(), tdesc.size() * 4);
  if (use_cb) {
    cp(c->col_pn, pl.col.data(), (size_t)nnz * 4);
    cp(c->val_pn, pl.val.data(), (size_t)nnz * 8);
    if (c->val32_pn) {
      std::vector<float> v32(pl.val.begin(), pl.val.end());
      cp(c->val32_pn, v32.data(), (size_t)nnz * 4);
    }
    cp(c->tiles_pn, pl.tiles.data(), pl.tiles.size() * 4);
    cp(c->toff_pn, pl.toff.data(), pl.toff.size() * 4);
    cp(c->off_pn, pl.off.data(), pl.off.size() * 2);
    cp(c->ptile, pl.ptile.data(), pl.ptile.size() * 4);
  }
  auto zero_pad = [&](void* p, size_t esz) {
    if (rc == RKS_OK && p && hipMemset((char*)p + (size_t)nnz * esz, 0, rks::kCsrPad * esz) != hipSuccess)
      rc = RKS_EHIP;
  };
  zero_pad(c->col, 4);
  zero_pad(c->val, 8);
  zero_pad(c->val32, 4);
  zero_pad(c->vidx, 1);
  zero_pad(c->col_pn, 4);
  zero_pad(c->val_pn, 8);
  zero_pad(c->val32_pn, 4);
  if (rc == RKS_OK && hipMemset(c->U_lo, 0, (size_t)c->ldu * (m + 1) * ebytes) != hipSuccess) rc = RKS_EHIP;
  // padding rows of U, w and xcur stay zero for the whole life of the context
  if (rc == RKS_OK && hipMemset(c->w, 0, (size_t)c->ldu * 8) != hipSuccess) rc = RKS_EHIP;
  if (rc == RKS_OK && pair && hipMemset(c->xcur, 0, (size_t)c->ldu * 8) != hipSuccess) rc = RKS_EHIP;
  if (rc == RKS_OK && hipMemset(c->E, 0, (size_t)(m + 1) * (m + 1) * 8) != hipSuccess) rc = RKS_EHIP;
  if (rc != RKS_OK) {
    free_all(c);
    delete c;
    return fail(nullptr, rc, "uploading the matrix");
  }
  auto& e = c->env;
  e.stream = stm;
  e.n = n;
  e.prec = o.precision;
  if (pair) {
    e.pair_hi = (const float*)c->U_lo;
    e.pair_lo = (int16_t*)((char*)c->U_lo + (size_t)c->ldu * (m + 1) * 4);
    e.xcur = c->xcur;
  }
  e.rp = c->rp;
  e.col = c->col;
  e.val = c->val;
  e.val32 = c->val32;
  e.vidx = c->vidx;
  e.vtab = c->vtab;
  if (use_sl) {
    e.sl = 1;
    e.nsl = (int)nsl;
    e.sl_off = c->sl_off;
    e.col_sl = c->col_sl;
    e.val_sl = c->val_sl;
    e.vidx_sl = c->vidx_sl;
    e.val32_sl = c->val32_sl;
    e.sl_pad0 = pad0 ? 1 : 0;
  }
  e.tiles = c->tiles;
  e.ntiles = ntiles;
  if (use_cb) {
    e.cb = 1;
    e.npanels = pl.npanels;
    e.rows_pp = (int)pl.rows_pp;
    e.col_pn = c->col_pn;
    e.val_pn = c->val_pn;
    e.val32_pn = c->val32_pn;
    e.tiles_pn = c->tiles_pn;
    e.toff_pn = c->toff_pn;
    e.off_pn = c->off_pn;
    e.ptile = c->ptile;
  }
  e.ldu = c->ldu;
  c->ks = o.method == RKS_METHOD_KS_CGS2;
  e.sp_kind = c->ks ? 2 : o.sketch_kind;
  e.sp.d = d;
  e.sp.zeta = o.zeta;
  e.sp.k0 = (uint32_t)o.sketch_seed;
  e.sp.k1 = (uint32_t)(o.sketch_seed >> 32);
  e.sp.scale = (o.sketch_kind == RKS_SKETCH_SPARSE) ? 1.0 / std::sqrt((double)o.zeta) : 1.0 / std::sqrt((double)d);
  if (c->ks) {  // no sketch: the update and start kernels accumulate one squared norm instead
    e.sp.d = 1;
    e.sp.scale = 1.0;
  }
  *out = c;
  return RKS_OK;
}

void rks_destroy(rks_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->env.stream);
  free_all(c);
  delete c;
}

int32_t rks_num_pairs(const rks_ctx* c) { return c ? c->kr : 0; }

int rks_solve(rks_ctx* c, const double* u0, int32_t u0_on_device, rks_stats* st) {
  if (!c) return RKS_EINVAL;
  c->err.clear();
  rks_stats local;
  if (!st) st = &local;
  std::memset(st, 0, sizeof(*st));
  c->st = st;
  const auto t0 = std::chrono::steady_clock::now();
  set_basis(c, c->o.precision);
  // (the pair basis runs one phase: its stored values carry 39 bits of
  // significand, which the verified FP64 residual does not need refined)
  const bool mixed = c->o.precision == RKS_PREC_V32 || c->o.precision == RKS_PREC_VBF16;
  const bool refine = mixed && c->o.refine;
  PhaseOut p1{};
  int rc;
  if (refine) {
    double rtol = c->o.refine_tol;
    if (rtol <= 0.0) rtol = (c->o.precision == RKS_PREC_V32) ? 1e-6 : 1e-3;
    rtol = std::max(rtol, c->o.resid_tol);
    const double etol = std::max(c->tol, rtol);
    const int cap = std::max(1, c->o.max_restarts / 2);
    rc = run_phase(c, u0, u0_on_device, etol, rtol, cap, 0, &p1);
    st->restarts_lo = p1.restarts;
    st->t_lo = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc == RKS_OK) {
      // the low-precision phase's FP64 residual, verified on the device when
      // its estimates stopped it (a verified stop already has it)
      double mr = p1.maxres;
      if (!(mr > 0.0)) rc = verified_max_resid(c, &mr);
      st->max_resid_lo = mr;
    }
    if (rc == RKS_OK) {
      // FP64 refinement from a fixed combination of the low-precision Schur vectors
      rc = refine_start(c);
      if (rc == RKS_OK) {
        PhaseOut p2{};
        st->refined = 1;
        const int left = std::max(1, c->o.max_restarts - p1.restarts);
        rc = run_phase(c, c->u0tmp, 1, c->tol, c->o.resid_tol, left, p1.restarts + 1, &p2);
        p2.restarts += p1.restarts + 1;
        p2.thost += p1.thost;
        p2.resid_checks += p1.resid_checks;
        p1 = p2;
      }
    }
  } else {
    rc = run_phase(c, u0, u0_on_device, c->tol, c->o.resid_tol, c->o.max_restarts, 0, &p1);
  }
  if (rc == RKS_OK) {
    if (hipStreamSynchronize(c->env.stream) != hipSuccess) rc = fail(c, RKS_EHIP, "stream synchronize");
    flush_events(c);
  }
  st->converged = (p1.reason == 1 || p1.reason == 2) ? 1 : 0;
  st->stop_reason = p1.reason;
  st->max_resid = p1.maxres;
  st->resid_checks = p1.resid_checks;
  st->restarts = p1.restarts;
  st->locked = c->q;
  st->keff = c->kr;
  st->spmv_layout = c->env.cb ? RKS_SPMV_COLUMN_BLOCKS : (c->env.sl ? RKS_SPMV_SLICED : RKS_SPMV_ROWS);
  st->a_distinct = c->a_distinct;
  st->keep = c->keep;
  st->max_est = p1.maxest;
  st->t_host = p1.thost;
  st->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  c->st = nullptr;
  if (rc) return rc;
  c->solved = true;
  if (p1.reason == 3) return fail(c, RKS_ENOTCONV, "stagnation: the estimates stopped falling");
  return p1.reason != 0 ? RKS_OK : fail(c, RKS_ENOTCONV, "max_restarts reached");
}

int rks_eigpairs(rks_ctx* c, double* lam_re, double* lam_im, double* X, int32_t X_on_device, double* resid) {
  if (!c) return RKS_EINVAL;
  if (!c->solved) return fail(c, RKS_ESTATE, "rks_eigpairs before a successful rks_solve");
  const int ke = c->kr;
  Packed P = pack_ritz(c);
  if (X || resid) {
    int rc = ensure_resid_scratch(c);
    if (rc) return rc;
    double* Xd = (X && X_on_device) ? X : c->Xr;
    std::vector<double> res(ke, 0.0);
    rc = device_residuals(c, P, Xd, res.data(), true);
    if (rc) return rc;
    if (X && !X_on_device)
      HIPCHK(c, hipMemcpyAsync(X, Xd, (size_t)c->n * ke * 8, hipMemcpyDeviceToHost, c->env.stream));
    HIPCHK(c, hipStreamSynchronize(c->env.stream));
    if (resid) std::memcpy(resid, res.data(), (size_t)ke * 8);
  }
  for (int i = 0; i < ke; ++i) {
    if (lam_re) lam_re[i] = P.lam[i].real();
    if (lam_im) lam_im[i] = P.lam[i].imag();
  }
  return RKS_OK;
}

int rks_sketch(rks_ctx* c, const double* x_dev, double* z_dev) {
  if (!c || !x_dev || !z_dev) return RKS_EINVAL;
  if (c->ks) return fail(c, RKS_EINVAL, "deterministic Krylov-Schur has no sketch");
  const int G = rks::launch_init(c->env, nullptr, x_dev, 0, 0, c->spart, 0, 0);
  rks::launch_reduce(c->env, c->spart, G, nullptr, 0, z_dev, nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->env.stream));
  return RKS_OK;
}

int rks_sketch_noalloc(int64_t n, int32_t d, int32_t sketch_kind, int32_t zeta, uint64_t sketch_seed,
                       const double* x_dev, double* z_dev, void* stream) {
  g_create_err.clear();
  if (!x_dev || !z_dev) return fail(nullptr, RKS_EINVAL, "x or z is NULL");
  if (n < 1 || n >= ((int64_t)1 << 40)) return fail(nullptr, RKS_EINVAL, "need 1 <= n < 2^40");
  if (d < 1 || d > rks::kMaxD)
    return fail(nullptr, RKS_EINVAL, "need 1 <= d <= 1024 (the fixed scratch holds 512 x 1024 partial sums)");
  if (sketch_kind != RKS_SKETCH_GAUSS && sketch_kind != RKS_SKETCH_SPARSE)
    return fail(nullptr, RKS_EINVAL, "sketch_kind");
  if (sketch_kind == RKS_SKETCH_SPARSE && (zeta < 1 || zeta > 8 || zeta > d))
    return fail(nullptr, RKS_EINVAL, "need 1 <= zeta <= min(8, d)");
  double* part = nullptr;
  const int sr = rks::scratch_address(&part);
  if (sr != 0) return fail(nullptr, RKS_EHIP, "resolving the device scratch array");
  rks::LaunchEnv e{};
  e.stream = (hipStream_t)stream;
  e.n = n;
  e.prec = 0;
  e.sp_kind = sketch_kind;
  e.sp.d = d;
  e.sp.zeta = zeta;
  e.sp.k0 = (uint32_t)sketch_seed;
  e.sp.k1 = (uint32_t)(sketch_seed >> 32);
  e.sp.scale = (sketch_kind == RKS_SKETCH_SPARSE) ? 1.0 / std::sqrt((double)zeta) : 1.0 / std::sqrt((double)d);
  rks::launch_sketch_scratch(e, x_dev, part, z_dev);
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(nullptr, RKS_EHIP, std::string("sketch launch -> ") + hipGetErrorString(he));
  return RKS_OK;
}

int rks_spmv_sketch(rks_ctx* c, const double* x_dev, double* w_dev, double* z_dev) {
  if (!c || !x_dev || !w_dev || !z_dev) return RKS_EINVAL;
  if (c->ks) return fail(c, RKS_EINVAL, "deterministic Krylov-Schur has no sketch");
  const int G = rks::launch_spmv_sketch(c->env, x_dev, w_dev, c->zpart, 1, 0);
  rks::launch_reduce(c->env, c->zpart, G, nullptr, 0, z_dev, nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->env.stream));
  return RKS_OK;
}

int rks_arnoldi(rks_ctx* c, const double* u0, int32_t u0_on_device) {
  if (!c) return RKS_EINVAL;
  c->err.clear();
  c->st = nullptr;
  int rb = set_basis(c, c->o.precision);
  if (rb) return rb;
  int rc = start(c, u0, u0_on_device);
  if (rc) return rc;
  rc = extend(c);
  if (rc) return rc;
  rc = pull_and_recover(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->env.stream));
  return RKS_OK;
}

int rks_get_state(rks_ctx* c, int32_t* ncols, double* B, double* S, double* U) {
  if (!c) return RKS_EINVAL;
  if (!c->have_state) return fail(c, RKS_ESTATE, "no decomposition yet");
  int rc = pull_state(c);
  if (rc) return rc;
  const int nc = c->j + 1;
  if (ncols) *ncols = nc;
  if (B) std::memcpy(B, c->hB, (size_t)(c->m + 1) * c->m * 8);
  if (S) std::memcpy(S, c->hS, (size_t)c->d * (c->m + 1) * 8);
  if (U) {
    const size_t colb = (size_t)c->ldu * c->vbytes;
    std::vector<unsigned char> buf(colb);
    std::vector<int16_t> lo(c->pair ? c->ldu : 0);
    auto bf16 = [](uint16_t h) {
      const uint32_t u = (uint32_t)h << 16;
      float f;
      std::memcpy(&f, &u, 4);
      return (double)f;
    };
    for (int l = 0; l <= c->m; ++l) {
      double* dst = U + (size_t)l * c->n;
      if (l >= nc) {
        std::fill(dst, dst + c->n, 0.0);
        continue;
      }
      HIPCHK(c, hipMemcpy(buf.data(), basis_col(c, l), colb, hipMemcpyDeviceToHost));
      if (c->pair)
        HIPCHK(c, hipMemcpy(lo.data(), c->env.lo_of(basis_col(c, l)), (size_t)c->ldu * 2, hipMemcpyDeviceToHost));
      const double s = c->hcs[l];
      for (int64_t i = 0; i < c->n; ++i) {
        double v;
        if (c->vbytes == 8) {
          std::memcpy(&v, &buf[i * 8], 8);
        } else if (c->vbytes == 4) {
          float f;
          std::memcpy(&f, &buf[i * 4], 4);
          v = f;
          if (c->pair) {  // the stored value hi + lo 2^-15 ulp(hi)
            uint32_t hb;
            std::memcpy(&hb, &f, 4);
            const int ex = (int)((hb >> 23) & 0xFFu);
            v += std::ldexp((double)lo[i], std::max(ex, 1) - 165);
          }
        } else {
          uint16_t h;
          std::memcpy(&h, &buf[i * 2], 2);
          v = bf16(h);
        }
        dst[i] = v * s;
      }
    }
  }
  return RKS_OK;
}

int rks_rotate(rks_ctx* c, int32_t in0, int32_t min, int32_t out0, int32_t kout, const double* Y) {
  if (!c || !Y) return RKS_EINVAL;
  if (in0 < 0 || min < 1 || in0 + min > c->m + 1 || out0 < 0 || kout < 1 || kout > rks::kRotMax ||
      out0 + kout > c->m + 1)
    return RKS_EINVAL;
  // the stored columns carry lazy scales: fold them into Y, then the
  // outputs are normalised columns (scale 1)
  HIPCHK(c, hipStreamSynchronize(c->env.stream));
  HIPCHK(c, hipMemcpy(c->hcs, c->cs, (size_t)(c->m + 1) * 8, hipMemcpyDeviceToHost));
  for (int o = 0; o < kout; ++o)
    for (int l = 0; l < min; ++l) c->hY[l + (size_t)o * min] = c->hcs[in0 + l] * Y[l + (size_t)o * min];
  for (int o = 0; o < kout; ++o) c->hcs[out0 + o] = 1.0;
  HIPCHK(c, hipMemcpy(c->Yd, c->hY, (size_t)min * kout * 8, hipMemcpyHostToDevice));
  rks::launch_rotate(c->env, c->U, c->ldu, in0, min, c->U, c->ldu, out0, kout, c->Yd, -1, 0, 0.0, 0);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->cs, c->hcs, (size_t)(c->m + 1) * 8, hipMemcpyHostToDevice, c->env.stream));
  HIPCHK(c, hipStreamSynchronize(c->env.stream));
  return RKS_OK;
}

int rks_copy_probe(const void* src, void* dst, int64_t nbytes, int32_t iters, double* gbs, void* stream) {
  if (!src || !dst || nbytes < 16 || nbytes % 16 != 0 || iters < 1 || !gbs) return RKS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return RKS_EHIP;
  rks::launch_copy16(st, src, dst, nbytes / 16);  // warm-up
  (void)hipEventRecord(a, st);
  for (int i = 0; i < iters; ++i) rks::launch_copy16(st, src, dst, nbytes / 16);
  (void)hipEventRecord(b, st);
  float ms = 0.f;
  const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!ok || ms <= 0.f) return RKS_EHIP;
  *gbs = 2.0 * (double)nbytes * iters / (ms * 1e-3) / 1e9;
  return RKS_OK;
}

int rks_read_probe(const void* src, int64_t nbytes, int32_t iters, double* gbs, void* stream) {
  if (!src || nbytes < 16 || nbytes % 16 != 0 || iters < 1 || !gbs) return RKS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return RKS_EHIP;
  rks::launch_read16(st, src, nbytes / 16);  // warm-up
  (void)hipEventRecord(a, st);
  for (int i = 0; i < iters; ++i) rks::launch_read16(st, src, nbytes / 16);
  (void)hipEventRecord(b, st);
  float ms = 0.f;
  const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!ok || ms <= 0.f) return RKS_EHIP;
  *gbs = (double)nbytes * iters / (ms * 1e-3) / 1e9;
  return RKS_OK;
}

int rks_host_schur(int32_t n, double* A, double* Z) {
  if (n < 1 || !A || !Z) return RKS_EINVAL;
  return rks::real_schur(n, A, n, Z, n) == 0 ? RKS_OK : RKS_EDENSE;
}

int rks_host_order(int32_t n, double* T, double* Z, int32_t which, int32_t kw, int32_t* p) {
  if (n < 1 || !T || !Z || !p || which < 0 || which > 3 || kw < 0) return RKS_EINVAL;
  int pp = 0;
  const int r = rks::order_wanted(n, T, n, Z, n, which, kw, &pp);
  *p = pp;
  return r == 0 ? RKS_OK : RKS_EDENSE;
}

}  // extern "C"
