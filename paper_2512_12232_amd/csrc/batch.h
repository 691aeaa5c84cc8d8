// Batched solves: many independent meshes (a delta-sweep of the same layout, uneven
// sizes) advanced together.  Part of solve.hip's translation unit.
//
// Every kernel covers all systems: its blocks are dealt to the systems through a block
// map (block b -> (system, virtual block); each system's blocks start at a multiple of
// 8, so the XCD-aware order of the single solve holds per system), and each system's
// arguments come from a per-system table in device memory.  The CG iteration is the
// one-kernel iteration of step.h: a replayed block of m launches reads its first
// launch index from each system's device state (jbase), the launch's offset in
// the block is a captured argument, so the launch sequence of a block is the same
// every time: it is captured once as a hipGraph and replayed until every system has
// stopped.  Systems that have stopped return at the top of every kernel.  jbase is odd
// at every replay, so the launches that update the iterate (odd indices) are the same
// captured launches every time.
//
// MFP_FP64: FP64 CG for every system (stopping on each system's own residual); a block
// is an even number m of launches and jbase advances by m.
// MFP_FP32_IR: FP32 CG for every system; a block is an odd number m of launches, so
// that its last launch J is odd and the FP32 correction is complete after it.  The
// correction is folded into the FP64 iterate, the residual is recomputed with the FP64
// apply, the stopping test is made on that FP64 residual, and launch J is run again as
// the first launch of the next block: a restart that forms p_J from the new residual
// and p_{J-1} with beta = |r_new|^2 / |r_{J-1}|^2, as the single solve's residual
// replacement does (jbase advances by m - 1).
#pragma once

namespace mfp {

struct BElem {
  long long n;
  const int8_t* tag;
  double* x64;          // FP64 iterate (free nodes)
  float* e32;           // mixed: FP32 correction since the last refinement
  const double* g;      // Dirichlet lifting
  double* w64;          // out: g + T x
  const double* q64;    // K w64
  float* r32;           // mixed: out, FP32 residual (parity slot 0)
  double* r64;          // FP64: out, residual (parity slot 0)
  double* spart;        // out: iteration-layout partials of the new residual (slot 0)
  double* part3;        // out: partials of q64.q64
  const double* bpart;  // body slots of the last plain apply
  const int* nslots;
  double* p64[2];       // FP64 directions by parity (completion of the iterate)
  float* p32[2];        // FP32 directions by parity
  DevState* out;        // mixed: FP64 body unknowns, refinement state
  DevState* in;         // CG state
  int G2;
  int nb;
};

// mode 0: w = g + T x (FP64 CG; body values of the current iterate);
// mode 1: x += e32, e32 = 0, then w with body values out->xb[0] + in->xb[iters & 1]
//         (the inner correction of the last launch).
__global__ void __launch_bounds__(BLOCK) k_b_formw(const BElem* __restrict__ bv,
                                                   const int2* __restrict__ map, int mode) {
  const int2 vm = map[blockIdx.x];
  const BElem& b = bv[vm.x];
  if (mode == 1 && b.out->done) return;
  const double* xbi = b.in->xb[b.in->iters & 1];
  const double* xbo = b.out->xb[0];
  for (long long e = vm.y * (long long)BLOCK + threadIdx.x; e < b.n;
       e += (long long)b.G2 * BLOCK) {
    double xv = b.x64[e];
    if (mode == 1) {
      xv += (double)b.e32[e];
      b.x64[e] = xv;
      b.e32[e] = 0.f;
    }
    const int8_t tg = b.tag[e];
    double v = 0.0;
    if (tg == TAG_FREE)
      v = xv;
    else if (tg == TAG_DIR)
      v = b.g[e];
    else if (tg >= TAG_BODY0)
      v = mode == 1 ? xbo[tg - TAG_BODY0] + xbi[tg - TAG_BODY0] : xbi[tg - TAG_BODY0];
    b.w64[e] = v;
  }
}

// r = -K w at free nodes (K w is zero elsewhere), per-block partials of r.r in the
// iteration layout (r.r, 0, 0, 0) in slot 0, and of (K w).(K w).
// mode 0 (FP64 start): r64; mode 1 (mixed refinement): r32 (rounded); mode 2 (FP64
// true residual): partials only.
__global__ void __launch_bounds__(BLOCK) k_b_resid(const BElem* __restrict__ bv,
                                                   const int2* __restrict__ map, int mode) {
  __shared__ double s_red[BLOCK / 64];
  const int2 vm = map[blockIdx.x];
  const BElem& b = bv[vm.x];
  if (mode == 1 && b.out->done) return;
  double a2 = 0.0, a3 = 0.0;
  for (long long e = vm.y * (long long)BLOCK + threadIdx.x; e < b.n;
       e += (long long)b.G2 * BLOCK) {
    const double q = b.q64[e];
    a3 += q * q;
    if (mode == 0) {
      b.r64[e] = -q;
      a2 += q * q;
    } else if (mode == 1) {
      const float v = (float)(-q);
      b.r32[e] = v;
      a2 += (double)v * (double)v;
    }
  }
  const double s2 = block_sum(a2, s_red);
  const double s3 = block_sum(a3, s_red);
  if (threadIdx.x < 4 && mode != 2) b.spart[4 * vm.y + threadIdx.x] = threadIdx.x == 0 ? s2 : 0.0;
  if (threadIdx.x == 0) b.part3[vm.y] = s3;
}

// One block per system; rr = |b - A x|^2 from the partials of (K w).(K w) and the body
// rows.  mode 0: FP64 start (fresh run from launch 1); mode 1: mixed refinement (init
// marks the first one): fold the body corrections, test the FP64 residual, and set up
// the restart of the block's last launch J (in->iters); mode 2: FP64 true residual.
// flags[v] = stop code.
__global__ void __launch_bounds__(BLOCK) k_b_fin(const BElem* __restrict__ bv, int mode, int init,
                                                 double rtol2, long long kmax_abs,
                                                 int* __restrict__ flags) {
  __shared__ double s_red[BLOCK / 64];
  __shared__ double s_qb[MFP_MAX_BODIES];
  const BElem& b = bv[blockIdx.x];
  DevState* in = b.in;
  DevState* out = b.out;
  if (mode == 1 && out->done) {
    if (threadIdx.x == 0) flags[blockIdx.x] = out->done;
    return;
  }
  body_sums(b.bpart, b.nslots, b.nb, s_qb);
  double s3 = 0.0;
  for (int i = threadIdx.x; i < b.G2; i += BLOCK) s3 += b.part3[i];
  s3 = block_sum(s3, s_red);
  if (threadIdx.x != 0) return;
  const int nb = b.nb;
  double rbr = 0.0;
  for (int k = 0; k < nb; ++k) {
    const double v = in->bb[k] - s_qb[k];
    rbr += v * v;
  }
  const double rr = s3 + rbr;
  auto fresh = [&]() {
    for (int k = 0; k < nb; ++k) in->pb[0][k] = 0.0;
    in->rr_prev = 0.0;
    in->stop_rel = 0.0;
    in->alpha_hist[0] = in->alpha_hist[1] = 0.0;
    in->jbase = 1;
    in->k0 = 1;
    in->iters = 0;
    in->kmax = kmax_abs;
  };
  if (mode == 0) {
    for (int k = 0; k < nb; ++k) in->rb[0][k] = in->bb[k] - s_qb[k];
    fresh();
    in->rr0 = rr;
    in->rr_stop = rtol2 * rr;
    in->done = rr > 0.0 ? 0 : 1;
    flags[blockIdx.x] = in->done;
    return;
  }
  if (mode == 2) {
    in->rr_true = rr;
    return;
  }
  // mixed refinement: fold the body corrections, record the FP64 residual
  const long long J = in->iters;
  for (int k = 0; k < nb; ++k) {
    out->xb[0][k] += in->xb[J & 1][k];
    in->xb[0][k] = 0.0;  // the correction restarts from zero
    in->xb[1][k] = 0.0;
  }
  out->rr_true = rr;
  if (init) {
    out->rr0 = rr;
    fresh();
    in->rr_stop = -1.0;  // the FP32 recursion never stops the solve by itself
    in->done = 0;
    out->outer_count = 0;
  } else {
    out->outer_count += 1;
  }
  int code = 0;
  if (!(rr == rr))
    code = 2;
  else if (rr <= rtol2 * out->rr0)
    code = 1;
  else if (in->done)
    code = in->done;
  out->iters = J;
  if (code) {
    out->done = code;
    in->done = code;
    for (int k = 0; k < nb; ++k) out->xb[1][k] = out->xb[0][k];
  } else if (init) {
    for (int k = 0; k < nb; ++k) in->rb[0][k] = in->bb[k] - s_qb[k];
  } else {
    // launch J again as a start: it reads slot (J-1)&1, where the new residual has
    // replaced r_{J-1} (k_b_resid) and p_{J-1} is kept
    const int prv = (int)((J - 1) & 1);
    for (int k = 0; k < nb; ++k) in->rb[prv][k] = in->bb[k] - s_qb[k];
    in->k0 = J;
    in->rr_prev = in->rr[prv];  // |r_{J-1}|^2
    in->alpha_hist[0] = in->alpha_hist[1] = 0.0;  // no direction pending in e
  }
  flags[blockIdx.x] = out->done;
}

// The iterate after the last launch J of each system (see k_finish): J = the launch
// that stopped, or jbase + off for a system still running (off = m - 1 inside a
// replay, -1 after the replays), whose x lacks alpha_{J-1} p_{J-1} when J is even
// (an odd J leaves it complete).  Block 0 of each system records J in iters.
// mode 1: FP32 correction of a mixed solve.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_b_finish(const BElem* __restrict__ bv,
                                                    const int2* __restrict__ map, int off,
                                                    int mode) {
  const int2 vm = map[blockIdx.x];
  const BElem& b = bv[vm.x];
  if (mode == 1 && b.out->done) return;
  DevState* in = b.in;
  const bool stopped = in->done != 0;
  const long long J = stopped ? in->iters : in->jbase + off;
  if (vm.y == 0 && threadIdx.x == 0) in->iters = J;  // same value if stopped
  if (!stopped && (J & 1)) return;
  T* x;
  const T* p0;
  const T* p1;
  if constexpr (sizeof(T) == 8) {
    x = b.x64;
    p0 = b.p64[0];
    p1 = b.p64[1];
  } else {
    x = b.e32;
    p0 = b.p32[0];
    p1 = b.p32[1];
  }
  const T a1 = (T)in->alpha;
  const bool two = ((J - 1) & 1) == 0;
  const T a2 = two ? (T)in->alpha_hist[(J - 1) & 1] : (T)0;
  const T* pa = ((J - 1) & 1) ? p1 : p0;
  const T* pb = (J & 1) ? p1 : p0;
  for (long long e = vm.y * (long long)BLOCK + threadIdx.x; e < b.n;
       e += (long long)b.G2 * BLOCK)
    x[e] = (x[e] + a2 * pb[e]) + a1 * pa[e];
}

// End of a replayed block: next block's first launch (adv = m, or m - 1 when the
// block's last launch is run again as a restart); FP64: flags[v] = stop code.
__global__ void k_b_advance(const BElem* __restrict__ bv, int nvar, int adv, int fp64,
                            int* __restrict__ flags) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvar) return;
  DevState* in = bv[v].in;
  if (!in->done) in->jbase += adv;
  if (fp64) flags[v] = in->done;
}

struct BatchPlan {
  int nvar = 0, nb = 0, precision = MFP_FP64;
  std::vector<SolveWs> w;
  std::vector<int> G, G2, GS;   // blocks: residual apply, streaming kernels, iteration
  int totG = 0, totG2 = 0, totGS = 0;
  ApplyArgs<double>* a64 = nullptr;   // plain FP64 apply (residuals)
  StepArgs<double>* s64 = nullptr;    // FP64 iteration
  StepArgs<float>* s32 = nullptr;     // FP32 iteration
  BElem* be = nullptr;
  int2* amap = nullptr;
  int2* umap = nullptr;
  int2* smap = nullptr;
  int* flags = nullptr;
  size_t bytes = 0;
};

// Tasks per wavefront segment (on average, by cost) in batched residual applies: the
// launch holds many systems, so segments are sized for the prefetch, not for residency.
constexpr int BATCH_SEG = 4;
// Tasks per wavefront of the batched iteration (its launch holds many systems, far more
// wavefronts than are resident).  Each wavefront's scalar phase (partials in, block
// sums, barriers) is a fixed latency, spread over its tasks; measured on the 256-system
// sweep (FP64 / FP32 + refinement, ms): 1 task 1647 / 1076, 2: 1424 / 929,
// 4: 1297 / 896, 8: 1286 / 910.
constexpr int BATCH_TPW = 4;

// Schedule of a batched solve: node rows per task (4 or 5), tasks per wavefront and
// the element mode (stored entries or geometry on the fly) of every system.  5-row
// tasks by default (256-system sweep, geometry on the fly, 4 tasks per wavefront:
// FP64 1270 -> 1244 ms, FP32 + refinement 890 -> 881 ms against 4-row tasks).
struct BatchSchedule {
  int hc = 5;
  int tpw = BATCH_TPW;
  int kst = 0;
  int ipl = 0;  // launches per replayed block when the caller passes 0 (0: 64)
};

// Built-in rule, then the tuning cache's batched entry (grid 0 x 0: one entry covers
// every batch of this precision on this device), then the caller's explicit fields.
static int resolve_batch_schedule(int precision, const mfp_solver_opts* o, BatchSchedule* out) {
  BatchSchedule bs;
  TuneEntry e;
  mfp_grid any{};
  if (tuned_entry(&any, precision, 1, &e)) {
    if (e.task_rows == 4 || e.task_rows == 5) bs.hc = e.task_rows;
    if (e.tasks_per_wave >= 1 && e.tasks_per_wave <= 64) bs.tpw = e.tasks_per_wave;
    if (e.element_mode == 1 || e.element_mode == 2) bs.kst = e.element_mode == 2;
    if (e.iters_per_launch >= 2 && e.iters_per_launch <= 1024) bs.ipl = e.iters_per_launch;
  }
  if (o) {
    if (o->element_mode < 0 || o->element_mode > 2 || o->batch_tasks_per_wave < 0 ||
        o->batch_tasks_per_wave > 64 ||
        (o->task_rows != 0 && o->task_rows != 4 && o->task_rows != 5)) {
      set_error("invalid batched schedule: task_rows 0, 4 or 5, element_mode 0..2, "
                "batch_tasks_per_wave 0..64");
      return MFP_E_ARG;
    }
    if (o->task_rows) bs.hc = o->task_rows;
    if (o->element_mode) bs.kst = o->element_mode == 2;
    if (o->batch_tasks_per_wave) bs.tpw = o->batch_tasks_per_wave;
  }
  *out = bs;
  return MFP_OK;
}

static int batch_step_blocks(const Layout& L, int tpw) {
  long long g = ((long long)L.ntasks() + WAVES * tpw - 1) / (WAVES * tpw);
  g = (g + 7) & ~7LL;
  if (g > 1024) g = 1024;
  return (int)g;
}

static size_t batch_layout(int nvar, const mfp_variant* v, int nb, int precision, void* base,
                           BatchPlan* P, const BatchSchedule& bs) {
  Schedule sc;
  sc.hc = bs.hc;
  sc.kst = bs.kst;
  Bump bp(base);
  if (P) {
    P->nvar = nvar;
    P->nb = nb;
    P->precision = precision;
    P->w.resize(nvar);
    P->G.resize(nvar);
    P->G2.resize(nvar);
    P->GS.resize(nvar);
  }
  int totG = 0, totG2 = 0, totGS = 0;
  for (int i = 0; i < nvar; ++i) {
    const size_t sz = solve_layout(&v[i].grid, nb, precision, nullptr, nullptr, &sc);
    char* b = bp.take<char>(sz);
    SolveWs w;
    solve_layout(&v[i].grid, nb, precision, b, &w, &sc);
    w.sp = seg_plan(w.L, (w.L.ntasks() + BATCH_SEG - 1) / BATCH_SEG);
    const int G = w.sp.G;
    const int G2 = grid_blocks(w.L.n);
    const int GS = batch_step_blocks(w.L, bs.tpw);
    if (P) {
      P->w[i] = w;
      P->G[i] = G;
      P->G2[i] = G2;
      P->GS[i] = GS;
    }
    totG += G;
    totG2 += G2;
    totGS += GS;
  }
  if (P) {
    P->totG = totG;
    P->totG2 = totG2;
    P->totGS = totGS;
  }
  auto a64 = bp.take<ApplyArgs<double>>(nvar);
  auto s64 = bp.take<StepArgs<double>>(nvar);
  auto s32 = bp.take<StepArgs<float>>(nvar);
  auto be = bp.take<BElem>(nvar);
  auto amap = bp.take<int2>(totG);
  auto umap = bp.take<int2>(totG2);
  auto smap = bp.take<int2>(totGS);
  auto flags = bp.take<int>(nvar);
  if (P) {
    P->a64 = a64;
    P->s64 = s64;
    P->s32 = s32;
    P->be = be;
    P->amap = amap;
    P->umap = umap;
    P->smap = smap;
    P->flags = flags;
    P->bytes = bp.off + 256;
  }
  return bp.off + 256;
}

// Arguments of a system's batched iteration: the single solve's arguments with the
// parity slots filled in and the launch index taken from the device state.
template <typename T>
static StepArgs<T> batch_step_args(const SolveWs& w, const mfp_grid& g, int nb, int GS,
                                   int npart0, const T* dx, const T* dy, T* r0, T* r1, T* p0,
                                   T* p1, T* q0, T* q1, T* x, DevState* st) {
  StepRun<T> run = make_step_run<T>(w, g, nb, dx, dy, r0, r1, p0, p1, q0, q1, x, st);
  StepArgs<T> a = run.a;
  a.G = GS;
  a.stream = 1;  // k_step_batch stores streaming
  a.npart0 = npart0;
  for (int s = 0; s < 2; ++s) {
    a.rs[s] = run.r[s];
    a.ps[s] = run.p[s];
    a.qs[s] = run.q[s];
    a.parts[s] = run.part[s];
    a.bparts[s] = run.bpart[s];
  }
  return a;
}

template <typename T, int HC>
static void launch_step_batch_k(int G, hipStream_t st, const StepArgs<T>* args,
                                const int2* map, int koff, int kst) {
  // launch jbase + koff is odd (jbase is odd) for even koff: those update the iterate
  if (kst) {
    if ((koff & 1) == 0)
      k_step_batch<T, HC, true, true><<<G, BLOCK, 0, st>>>(args, map, koff);
    else
      k_step_batch<T, HC, false, true><<<G, BLOCK, 0, st>>>(args, map, koff);
  } else {
    if ((koff & 1) == 0)
      k_step_batch<T, HC, true, false><<<G, BLOCK, 0, st>>>(args, map, koff);
    else
      k_step_batch<T, HC, false, false><<<G, BLOCK, 0, st>>>(args, map, koff);
  }
}

template <typename T>
static void launch_step_batch(int G, hipStream_t st, const StepArgs<T>* args, const int2* map,
                              int koff, const BatchSchedule& bs) {
  if (bs.hc == 5)
    launch_step_batch_k<T, 5>(G, st, args, map, koff, bs.kst);
  else
    launch_step_batch_k<T, 4>(G, st, args, map, koff, bs.kst);
}

// The FP64 residual apply of every system (the layouts' task rows).
static void launch_apply_batch(int G, hipStream_t st, const ApplyArgs<double>* args,
                               const int2* map, const BatchSchedule& bs) {
  if (bs.hc == 5)
    k_apply_batch<double, 5><<<G, BLOCK, 0, st>>>(args, map);
  else
    k_apply_batch<double, 4><<<G, BLOCK, 0, st>>>(args, map);
}

}  // namespace mfp

extern "C" size_t mfp_batched_workspace_size_opts(int32_t nvar, const mfp_variant* vars_h,
                                                  int32_t nbody, const mfp_solver_opts* opts) {
  if (nvar < 1 || !vars_h || !opts || nbody < 0 || nbody > MFP_MAX_BODIES) return 0;
  for (int i = 0; i < nvar; ++i)
    if (vars_h[i].grid.nx < 2 || vars_h[i].grid.ny < 2) return 0;
  mfp::BatchSchedule bs;
  if (mfp::resolve_batch_schedule(opts->precision, opts, &bs) != MFP_OK) return 0;
  return mfp::batch_layout(nvar, vars_h, nbody, opts->precision, nullptr, nullptr, bs);
}

extern "C" size_t mfp_batched_workspace_size(int32_t nvar, const mfp_variant* vars_h,
                                             int32_t nbody, int32_t precision) {
  mfp_solver_opts o{};
  o.precision = precision;
  return mfp_batched_workspace_size_opts(nvar, vars_h, nbody, &o);
}

extern "C" int mfp_psi_solve_batched(int32_t nvar, const mfp_variant* vars_h,
                                     const mfp_circle* circles_h, int32_t nbody,
                                     const mfp_flow* flow, const mfp_solver_opts* opts,
                                     int32_t iters_per_launch, int32_t pair_lo, int32_t pair_hi,
                                     double* psi_b_h, double* copfi_h, mfp_stats* stats_h,
                                     void* ws, size_t ws_bytes, void* stream_) {
  using namespace mfp;
  clear_error();
  if (nvar < 1 || !vars_h || !flow || !opts || !ws || (nbody > 0 && (!circles_h || !psi_b_h))) {
    set_error("bad argument");
    return MFP_E_ARG;
  }
  if (opts->precision != MFP_FP64 && opts->precision != MFP_FP32_IR) {
    set_error("batched solves take MFP_FP64 or MFP_FP32_IR");
    return MFP_E_ARG;
  }
  if (!(opts->rtol > 0.0) || opts->kmax < 1 || opts->psi0) {
    set_error("rtol must be > 0, kmax >= 1, no warm start");
    return MFP_E_ARG;
  }
  if (pair_lo >= nbody || pair_hi >= nbody) {
    set_error("pair index out of range");
    return MFP_E_ARG;
  }
  for (int i = 0; i < nvar; ++i) {
    MFP_TRY(check_solve_args(&vars_h[i].grid, circles_h + (size_t)i * nbody, nbody,
                             vars_h[i].disp, vars_h[i].kind, vars_h[i].body, flow, opts, ws));
  }
  BatchSchedule bs;
  MFP_TRY(resolve_batch_schedule(opts->precision, opts, &bs));
  const size_t need = batch_layout(nvar, vars_h, nbody, opts->precision, nullptr, nullptr, bs);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  BatchPlan P;
  batch_layout(nvar, vars_h, nbody, opts->precision, ws, &P, bs);
  const int nb = nbody;
  const bool mixed = opts->precision == MFP_FP32_IR;
  // launches per replay: FP64 an even number (jbase advances by m), mixed an odd one
  // (its last launch is run again as the restart: jbase advances by m - 1), so that
  // jbase stays odd and every replay has the same launch parities (the captured
  // kernel instances depend on them)
  int m = iters_per_launch > 0 ? iters_per_launch : (bs.ipl > 0 ? bs.ipl : 64);
  m += m & 1;
  // an unrefined FP32 run loses its accuracy (and can break down) after a few hundred
  // iterations
  if (mixed && m > 256) m = 256;
  if (mixed) m += 1;
  const int adv = mixed ? m - 1 : m;
  const double rtol2 = opts->rtol * opts->rtol;

  // per-system setup and argument tables
  std::vector<ApplyArgs<double>> ha64(nvar);
  std::vector<StepArgs<double>> hs64(nvar);
  std::vector<StepArgs<float>> hs32(nvar);
  std::vector<BElem> hbe(nvar);
  std::vector<int2> hamap, humap, hsmap;
  hamap.reserve(P.totG);
  humap.reserve(P.totG2);
  hsmap.reserve(P.totGS);
  const long long kmax_abs = 1 + opts->kmax;
  for (int i = 0; i < nvar; ++i) {
    const mfp_grid& g = vars_h[i].grid;
    const SolveWs& w = P.w[i];
    const mfp_circle* ci = circles_h + (size_t)i * nb;
    MFP_TRY(setup(g, ci, nb, vars_h[i].disp, vars_h[i].body, flow, opts->precision, w, st));
    MFP_TRY_HIP(hipMemcpyAsync(&w.nslots_h, w.nslots, sizeof(int), hipMemcpyDeviceToHost, st));
    MFP_TRY_HIP(hipStreamSynchronize(st));  // slot count
    const int G = P.G[i], G2 = P.G2[i], GS = P.GS[i];
    for (int b = 0; b < G; ++b) hamap.push_back(make_int2(i, b));
    for (int b = 0; b < G2; ++b) humap.push_back(make_int2(i, b));
    for (int b = 0; b < GS; ++b) hsmap.push_back(make_int2(i, b));
    // plain FP64 apply on w (residuals)
    ApplyArgs<double> a = make_apply_args<double>(w, g, nb, w.dx, w.dy);
    a.src = w.p0;
    a.q = w.q;
    a.skip = mixed ? &w.st->done : nullptr;
    ha64[i] = a;
    if (mixed)
      hs32[i] = batch_step_args<float>(w, g, nb, GS, G2, w.dxf, w.dyf, w.rf, w.r1f, w.p0f, w.p1f,
                                       w.qf, w.q1f, w.xf, w.st2);
    else
      hs64[i] = batch_step_args<double>(w, g, nb, GS, G2, w.dx, w.dy, w.r, w.r1, w.p0, w.p1, w.q,
                                        w.q1, w.x, w.st);
    BElem be{};
    be.n = w.L.n;
    be.tag = w.tag;
    be.x64 = w.x;
    be.e32 = mixed ? w.xf : nullptr;
    be.g = w.g;
    be.w64 = w.p0;
    be.q64 = w.q;
    be.r32 = mixed ? w.rf : nullptr;
    be.r64 = w.r;
    be.spart = w.spart;
    be.part3 = w.part3;
    be.bpart = w.bpart;
    be.nslots = w.nslots;
    be.p64[0] = w.p0;
    be.p64[1] = w.p1;
    be.p32[0] = mixed ? w.p0f : nullptr;
    be.p32[1] = mixed ? w.p1f : nullptr;
    be.out = w.st;
    be.in = mixed ? w.st2 : w.st;
    be.G2 = G2;
    be.nb = nb;
    hbe[i] = be;
  }
  MFP_TRY_HIP(hipMemcpyAsync(P.a64, ha64.data(), sizeof(ApplyArgs<double>) * nvar, hipMemcpyHostToDevice, st));
  if (mixed)
    MFP_TRY_HIP(hipMemcpyAsync(P.s32, hs32.data(), sizeof(StepArgs<float>) * nvar, hipMemcpyHostToDevice, st));
  else
    MFP_TRY_HIP(hipMemcpyAsync(P.s64, hs64.data(), sizeof(StepArgs<double>) * nvar, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.be, hbe.data(), sizeof(BElem) * nvar, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.amap, hamap.data(), sizeof(int2) * hamap.size(), hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.umap, humap.data(), sizeof(int2) * humap.size(), hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.smap, hsmap.data(), sizeof(int2) * hsmap.size(), hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));  // host tables above

  hipEvent_t e0, e1;
  MFP_TRY_HIP(hipEventCreate(&e0));
  MFP_TRY_HIP(hipEventCreate(&e1));
  MFP_TRY_HIP(hipEventRecord(e0, st));
  // start: residual of x = 0 for every system
  k_b_formw<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, mixed ? 1 : 0);
  launch_apply_batch(P.totG, st, P.a64, P.amap, bs);
  k_b_resid<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, mixed ? 1 : 0);
  k_b_fin<<<nvar, BLOCK, 0, st>>>(P.be, mixed ? 1 : 0, 1, rtol2, kmax_abs, P.flags);
  MFP_TRY_HIP(hipGetLastError());

  // capture m iterations (+ the FP64 refinement) once, replay until all systems stop
  hipStream_t cs;
  MFP_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int status = MFP_OK;
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    for (int k = 0; k < m; ++k) {
      if (mixed)
        launch_step_batch<float>(P.totGS, cs, P.s32, P.smap, k, bs);
      else
        launch_step_batch<double>(P.totGS, cs, P.s64, P.smap, k, bs);
    }
    if (mixed) {
      k_b_finish<float><<<P.totG2, BLOCK, 0, cs>>>(P.be, P.umap, m - 1, 1);
      k_b_formw<<<P.totG2, BLOCK, 0, cs>>>(P.be, P.umap, 1);
      launch_apply_batch(P.totG, cs, P.a64, P.amap, bs);
      k_b_resid<<<P.totG2, BLOCK, 0, cs>>>(P.be, P.umap, 1);
      k_b_fin<<<nvar, BLOCK, 0, cs>>>(P.be, 1, 0, rtol2, kmax_abs, P.flags);
    }
    k_b_advance<<<(nvar + 255) / 256, 256, 0, cs>>>(P.be, nvar, adv, mixed ? 0 : 1, P.flags);
    he = hipStreamEndCapture(cs, &graph);
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    set_error("graph capture: %s", hipGetErrorString(he));
    status = MFP_E_HIP;
  }
  std::vector<int> hflags(nvar, 0);
  long long launches = 0;
  const long long max_launches = (opts->kmax + adv - 1) / adv + 1;
  while (status == MFP_OK) {
    he = hipGraphLaunch(exec, st);
    if (he == hipSuccess) he = hipMemcpyAsync(hflags.data(), P.flags, sizeof(int) * nvar, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
      set_error("graph launch: %s", hipGetErrorString(he));
      status = MFP_E_HIP;
      break;
    }
    ++launches;
    bool all = true;
    for (int f : hflags) all = all && f != 0;
    if (all || launches >= max_launches) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  if (status != MFP_OK) return status;
  MFP_TRY_HIP(hipEventRecord(e1, st));
  if (!mixed) {
    // complete the iterates, then the true residual of every system
    k_b_finish<double><<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, -1, 0);
    k_b_formw<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, 0);
    launch_apply_batch(P.totG, st, P.a64, P.amap, bs);
    k_b_resid<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, 2);
    k_b_fin<<<nvar, BLOCK, 0, st>>>(P.be, 2, 0, rtol2, kmax_abs, P.flags);
    MFP_TRY_HIP(hipGetLastError());
  }
  // outputs
  std::vector<DevState> hs(nvar);
  for (int i = 0; i < nvar; ++i) {
    const mfp_grid& g = vars_h[i].grid;
    const SolveWs& w = P.w[i];
    const mfp_circle* ci = circles_h + (size_t)i * nb;
    double ylo = 0, yhi = 0;
    if (pair_lo >= 0 && pair_hi >= 0) {
      ylo = ci[pair_lo].cy;
      yhi = ci[pair_hi].cy;
    }
    if (vars_h[i].psi) {
      const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
      k_output<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, w.x, w.g, w.st,
                                                   vars_h[i].psi, pair_lo, pair_hi, flow->U,
                                                   ylo, yhi);
    }
    MFP_TRY_HIP(hipMemcpyAsync(&hs[i], w.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
  }
  MFP_TRY_HIP(hipGetLastError());
  MFP_TRY_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int worst = MFP_OK;
  for (int i = 0; i < nvar; ++i) {
    const DevState& s = hs[i];
    const long long J = s.iters;
    const double* xb = s.xb[J & 1];
    for (int b = 0; b < nb; ++b) psi_b_h[(size_t)i * nb + b] = xb[b];
    if (copfi_h && pair_lo >= 0 && pair_hi >= 0) {
      const mfp_circle* ci = circles_h + (size_t)i * nb;
      copfi_h[i] = (xb[pair_hi] - xb[pair_lo]) / (flow->U * (ci[pair_hi].cy - ci[pair_lo].cy));
    }
    const int code = s.done;
    if (code == 2) worst = MFP_E_BREAKDOWN;
    if ((code == 3 || code == 0) && worst == MFP_OK) worst = MFP_W_NOCONV;
    if (stats_h) {
      mfp_stats& o = stats_h[i];
      std::memset(&o, 0, sizeof(o));
      // CG steps: launches 2..J (a restart runs launch J again, without a step)
      o.iters = J > 1 ? J - 1 : 0;
      o.outer_iters = mixed ? s.outer_count : 0;
      o.inner_iters = mixed ? o.iters : 0;
      // element applies: the steps, the restarts and the FP64 residuals
      o.applies = o.iters + (mixed ? 2 * s.outer_count + 1 : 2);
      o.rnorm0 = std::sqrt(s.rr0);
      o.relres_true = s.rr0 > 0 ? std::sqrt(s.rr_true / s.rr0) : 0.0;
      o.solve_ms = ms;
      o.n_tiles = P.w[i].L.ntasks();
    }
  }
  if (stats_h) {
    // N_dof per system
    for (int i = 0; i < nvar; ++i) {
      long long nfree = 0;
      MFP_TRY_HIP(hipMemcpyAsync(&nfree, P.w[i].nfree, sizeof(long long), hipMemcpyDeviceToHost, st));
      MFP_TRY_HIP(hipStreamSynchronize(st));
      stats_h[i].n_free = nfree;
      stats_h[i].n_dof = nfree + nb;
    }
  }
  if (worst == MFP_E_BREAKDOWN) set_error("CG breakdown in at least one system");
  if (worst == MFP_W_NOCONV) set_error("at least one system reached kmax");
  return worst;
}
