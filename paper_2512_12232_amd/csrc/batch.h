// Batched solves: many independent meshes (a delta-sweep of the same layout, uneven
// sizes) advanced together.  Part of solve.hip's translation unit.
//
// Every kernel covers all systems: its blocks are dealt to the systems in proportion
// to their size through a block map (block b -> (system, virtual block)), and each
// system's arguments come from a per-system table in device memory.  The CG iteration
// index and the parity of the direction buffers live in each system's device state,
// so the launch sequence of a fixed number of iterations is the same every time: it
// is captured once as a hipGraph and replayed until every system has stopped.
// Systems that have stopped return at the top of every kernel.
//
// MFP_FP64: plain FP64 CG for every system (stopping on each system's own residual).
// MFP_FP32_IR: FP32 CG for every system; after each captured block of iterations
// the FP32 correction is folded into the FP64 iterate, the residual is recomputed
// with the FP64 apply and replaces the FP32 residual (the direction is kept), and the
// stopping test is made on that FP64 residual.
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
  float* r32;           // mixed: out, FP32 residual
  double* r64;          // FP64: out, residual
  double* part2;        // out: partials of the new residual norm^2 (r32 or r64)
  double* part3;        // out: partials of q64.q64
  const double* bpart;  // body slots of the last plain apply
  const int* nslots;
  DevState* out;        // mixed: FP64 body unknowns, refinement state
  DevState* in;         // CG state
  int G2;
  int nb;
};

// mode 0: w = g + T x (FP64 CG; body values of the current iterate);
// mode 1: x += e32, e32 = 0, then w with body values out->xb[0] + in->xb[ka & 1].
__global__ void __launch_bounds__(BLOCK) k_b_formw(const BElem* __restrict__ bv,
                                                   const int2* __restrict__ map, int mode) {
  const int2 vm = map[blockIdx.x];
  const BElem& b = bv[vm.x];
  if (mode == 1 && b.out->done) return;
  const double* xbi = mode == 1 ? b.in->xb[b.in->ka & 1] : b.in->xb[b.in->iters & 1];
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

// mode 0 (FP64 start): r64 = -q64, partials of r64^2 into part2 (and part3);
// mode 1 (mixed refinement): r32 = -q64 rounded, partials of r32^2 (part2) and
//   q64^2 (part3);
// mode 2 (FP64 true residual): partials of q64^2 into part3 only.
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
  if (threadIdx.x == 0) {
    b.part2[vm.y] = s2;
    b.part3[vm.y] = s3;
  }
}

// One block per system.  mode 0: FP64 CG start; mode 1: mixed refinement (init
// marks the first one); mode 2: FP64 true residual.  flags[v] = stop code.
__global__ void __launch_bounds__(BLOCK) k_b_fin(const BElem* __restrict__ bv, int mode, int init,
                                                 double rtol2, int* __restrict__ flags) {
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
  double s2 = 0.0, s3 = 0.0;
  for (int i = threadIdx.x; i < b.G2; i += BLOCK) {
    s2 += b.part2[i];
    s3 += b.part3[i];
  }
  s2 = block_sum(s2, s_red);
  s3 = block_sum(s3, s_red);
  if (threadIdx.x != 0) return;
  const int nb = b.nb;
  double rbr = 0.0;
  for (int k = 0; k < nb; ++k) {
    const double v = in->bb[k] - s_qb[k];
    rbr += v * v;
  }
  if (mode == 0) {
    for (int k = 0; k < nb; ++k) {
      in->rb[0][k] = in->bb[k] - s_qb[k];
      in->pb[1][k] = 0.0;
    }
    in->rb_rr[0] = rbr;
    in->rr[1] = 1.0;
    in->rr0 = s2 + rbr;
    in->rr_stop = rtol2 * in->rr0;
    in->iters = 0;
    in->ka = 0;
    in->done = in->rr0 > 0.0 ? 0 : 1;
    flags[blockIdx.x] = in->done;
    return;
  }
  if (mode == 2) {
    in->rr_true = s3 + rbr;
    return;
  }
  // mixed refinement: fold the body corrections, record the FP64 residual
  const int slot = (int)(in->ka & 1);
  for (int k = 0; k < nb; ++k) {
    out->xb[0][k] += in->xb[slot][k];
    in->xb[slot][k] = 0.0;
  }
  const double rr = s3 + rbr;
  out->rr_true = rr;
  if (init) {
    out->rr0 = rr;
    for (int k = 0; k < nb; ++k) in->pb[1][k] = 0.0;
    in->rr[1] = 1.0;
    in->ka = 0;
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
  if (code) {
    out->done = code;
    in->done = code;
    out->iters = in->ka;
    for (int k = 0; k < nb; ++k) out->xb[1][k] = out->xb[0][k];
  } else {
    for (int k = 0; k < nb; ++k) in->rb[slot][k] = in->bb[k] - s_qb[k];
    in->rb_rr[slot] = rbr;
  }
  flags[blockIdx.x] = out->done;
}

// FP64 CG: flags[v] = stop code of system v.
__global__ void k_b_flags(const BElem* __restrict__ bv, int nvar, int* __restrict__ flags) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nvar) flags[v] = bv[v].in->done;
}

struct BatchPlan {
  int nvar = 0, nb = 0, hc = 4, precision = MFP_FP64;
  std::vector<SolveWs> w;
  std::vector<int> G, G2;
  int totG = 0, totG2 = 0;
  ApplyArgs<float>* a32 = nullptr;
  UpdArgs<float>* u32 = nullptr;
  ApplyArgs<double>* a64 = nullptr;   // plain FP64 apply (residuals)
  ApplyArgs<double>* af64 = nullptr;  // fused FP64 apply (FP64 CG)
  UpdArgs<double>* u64 = nullptr;
  BElem* be = nullptr;
  int2* amap = nullptr;
  int2* umap = nullptr;
  int* flags = nullptr;
  size_t bytes = 0;
};

// Tasks per wavefront segment (on average, by cost) in batched applies: the launch
// holds many systems, so segments are sized for the prefetch, not for residency.
constexpr int BATCH_SEG = 4;

static int batch_hc(int nvar, const mfp_variant* v) {
  int hc = 4;
  for (int i = 0; i < nvar; ++i)
    if (make_layout(v[i].grid.nx, v[i].grid.ny).hc == 8) hc = 8;
  return hc;
}

static size_t batch_layout(int nvar, const mfp_variant* v, int nb, int precision, void* base,
                           BatchPlan* P) {
  Bump bp(base);
  const int hc = batch_hc(nvar, v);
  if (P) {
    P->nvar = nvar;
    P->nb = nb;
    P->hc = hc;
    P->precision = precision;
    P->w.resize(nvar);
    P->G.resize(nvar);
    P->G2.resize(nvar);
  }
  int totG = 0, totG2 = 0;
  for (int i = 0; i < nvar; ++i) {
    const size_t sz = solve_layout(&v[i].grid, nb, precision, nullptr, nullptr, hc);
    char* b = bp.take<char>(sz);
    SolveWs w;
    solve_layout(&v[i].grid, nb, precision, b, &w, hc);
    w.sp = seg_plan(w.L, (w.L.ntasks() + BATCH_SEG - 1) / BATCH_SEG);
    const int G = w.sp.G;
    const int G2 = grid_blocks(w.L.n);
    if (P) {
      P->w[i] = w;
      P->G[i] = G;
      P->G2[i] = G2;
    }
    totG += G;
    totG2 += G2;
  }
  if (P) {
    P->totG = totG;
    P->totG2 = totG2;
  }
  auto a32 = bp.take<ApplyArgs<float>>(nvar);
  auto u32 = bp.take<UpdArgs<float>>(nvar);
  auto a64 = bp.take<ApplyArgs<double>>(nvar);
  auto af64 = bp.take<ApplyArgs<double>>(nvar);
  auto u64 = bp.take<UpdArgs<double>>(nvar);
  auto be = bp.take<BElem>(nvar);
  auto amap = bp.take<int2>(totG);
  auto umap = bp.take<int2>(totG2);
  auto flags = bp.take<int>(nvar);
  if (P) {
    P->a32 = a32;
    P->u32 = u32;
    P->a64 = a64;
    P->af64 = af64;
    P->u64 = u64;
    P->be = be;
    P->amap = amap;
    P->umap = umap;
    P->flags = flags;
    P->bytes = bp.off + 256;
  }
  return bp.off + 256;
}

template <typename T>
static void launch_apply_batch(int hc, int G, hipStream_t st, const ApplyArgs<T>* args,
                               const int2* map, bool fused) {
  if (hc == 4) {
    if (fused)
      k_apply_batch<T, true, 4><<<G, BLOCK, 0, st>>>(args, map);
    else
      k_apply_batch<T, false, 4><<<G, BLOCK, 0, st>>>(args, map);
  } else {
    if (fused)
      k_apply_batch<T, true, 8><<<G, BLOCK, 0, st>>>(args, map);
    else
      k_apply_batch<T, false, 8><<<G, BLOCK, 0, st>>>(args, map);
  }
}

}  // namespace mfp

extern "C" size_t mfp_batched_workspace_size(int32_t nvar, const mfp_variant* vars_h,
                                             int32_t nbody, int32_t precision) {
  if (nvar < 1 || !vars_h || nbody < 0 || nbody > MFP_MAX_BODIES) return 0;
  for (int i = 0; i < nvar; ++i)
    if (vars_h[i].grid.nx < 2 || vars_h[i].grid.ny < 2) return 0;
  return mfp::batch_layout(nvar, vars_h, nbody, precision, nullptr, nullptr);
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
  const size_t need = batch_layout(nvar, vars_h, nbody, opts->precision, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  BatchPlan P;
  batch_layout(nvar, vars_h, nbody, opts->precision, ws, &P);
  const int nb = nbody;
  const bool mixed = opts->precision == MFP_FP32_IR;
  const int m = iters_per_launch > 0 ? iters_per_launch : 64;
  const double rtol2 = opts->rtol * opts->rtol;

  // per-system setup and argument tables
  std::vector<ApplyArgs<float>> ha32(nvar);
  std::vector<UpdArgs<float>> hu32(nvar);
  std::vector<ApplyArgs<double>> ha64(nvar), haf64(nvar);
  std::vector<UpdArgs<double>> hu64(nvar);
  std::vector<BElem> hbe(nvar);
  std::vector<int2> hamap, humap;
  hamap.reserve(P.totG);
  humap.reserve(P.totG2);
  for (int i = 0; i < nvar; ++i) {
    const mfp_grid& g = vars_h[i].grid;
    const SolveWs& w = P.w[i];
    const mfp_circle* ci = circles_h + (size_t)i * nb;
    MFP_TRY(setup(g, ci, nb, vars_h[i].disp, vars_h[i].body, flow, opts->precision, w, st));
    long long kmax = opts->kmax;
    MFP_TRY_HIP(hipMemcpyAsync(&w.st->kmax, &kmax, sizeof(long long), hipMemcpyHostToDevice, st));
    MFP_TRY_HIP(hipMemcpyAsync(&w.st2->kmax, &kmax, sizeof(long long), hipMemcpyHostToDevice, st));
    MFP_TRY_HIP(hipStreamSynchronize(st));  // kmax is a stack value
    const int G = P.G[i], G2 = P.G2[i];
    for (int b = 0; b < G; ++b) hamap.push_back(make_int2(i, b));
    for (int b = 0; b < G2; ++b) humap.push_back(make_int2(i, b));
    // plain FP64 apply on w (residuals)
    ApplyArgs<double> a = make_apply_args<double>(w, g, nb, w.dx, w.dy);
    a.src = w.p0;
    a.q = w.q;
    a.G = G;
    a.skip = mixed ? &w.st->done : nullptr;
    ha64[i] = a;
    // fused FP64 CG apply
    ApplyArgs<double> af = make_apply_args<double>(w, g, nb, w.dx, w.dy);
    af.r = w.r;
    af.q = w.q;
    af.part2 = w.part2;
    af.G2 = G2;
    af.G = G;
    af.kdev = 1;
    af.pbuf0 = w.p0;
    af.pbuf1 = w.p1;
    haf64[i] = af;
    UpdArgs<double> u{};
    u.n = w.L.n;
    u.x = w.x;
    u.r = w.r;
    u.q = w.q;
    u.part = w.part;
    u.G = G;
    u.bpart = w.bpart;
    u.nslots = w.nslots;
    u.part2 = w.part2;
    u.st = w.st;
    u.nb = nb;
    u.G2 = G2;
    u.kdev = 1;
    u.pbuf0 = w.p0;
    u.pbuf1 = w.p1;
    hu64[i] = u;
    if (mixed) {
      ApplyArgs<float> a3 = make_apply_args<float>(w, g, nb, w.dxf, w.dyf);
      a3.r = w.rf;
      a3.q = w.qf;
      a3.part2 = w.part2;
      a3.G2 = G2;
      a3.G = G;
      a3.kdev = 1;
      a3.pbuf0 = w.p0f;
      a3.pbuf1 = w.p1f;
      a3.st = w.st2;
      ha32[i] = a3;
      UpdArgs<float> u3{};
      u3.n = w.L.n;
      u3.x = w.xf;
      u3.r = w.rf;
      u3.q = w.qf;
      u3.part = w.part;
      u3.G = G;
      u3.bpart = w.bpart;
      u3.nslots = w.nslots;
      u3.part2 = w.part2;
      u3.st = w.st2;
      u3.nb = nb;
      u3.G2 = G2;
      u3.kdev = 1;
      u3.pbuf0 = w.p0f;
      u3.pbuf1 = w.p1f;
      hu32[i] = u3;
    }
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
    be.part2 = w.part2;
    be.part3 = w.part3;
    be.bpart = w.bpart;
    be.nslots = w.nslots;
    be.out = w.st;
    be.in = mixed ? w.st2 : w.st;
    be.G2 = G2;
    be.nb = nb;
    hbe[i] = be;
  }
  MFP_TRY_HIP(hipMemcpyAsync(P.a64, ha64.data(), sizeof(ApplyArgs<double>) * nvar, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.af64, haf64.data(), sizeof(ApplyArgs<double>) * nvar, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.u64, hu64.data(), sizeof(UpdArgs<double>) * nvar, hipMemcpyHostToDevice, st));
  if (mixed) {
    MFP_TRY_HIP(hipMemcpyAsync(P.a32, ha32.data(), sizeof(ApplyArgs<float>) * nvar, hipMemcpyHostToDevice, st));
    MFP_TRY_HIP(hipMemcpyAsync(P.u32, hu32.data(), sizeof(UpdArgs<float>) * nvar, hipMemcpyHostToDevice, st));
  }
  MFP_TRY_HIP(hipMemcpyAsync(P.be, hbe.data(), sizeof(BElem) * nvar, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.amap, hamap.data(), sizeof(int2) * hamap.size(), hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(P.umap, humap.data(), sizeof(int2) * humap.size(), hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));  // host tables above

  hipEvent_t e0, e1;
  MFP_TRY_HIP(hipEventCreate(&e0));
  MFP_TRY_HIP(hipEventCreate(&e1));
  MFP_TRY_HIP(hipEventRecord(e0, st));
  // start: residual of x = 0 for every system
  k_b_formw<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, mixed ? 1 : 0);
  launch_apply_batch<double>(P.hc, P.totG, st, P.a64, P.amap, false);
  k_b_resid<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, mixed ? 1 : 0);
  k_b_fin<<<nvar, BLOCK, 0, st>>>(P.be, mixed ? 1 : 0, 1, rtol2, P.flags);
  MFP_TRY_HIP(hipGetLastError());
  if (!mixed)
    for (int i = 0; i < nvar; ++i)
      MFP_TRY_HIP(hipMemsetAsync(P.w[i].p0, 0, sizeof(double) * P.w[i].L.n, st));

  // capture m iterations (+ the FP64 refinement) once, replay until all systems stop
  hipStream_t cs;
  MFP_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int status = MFP_OK;
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    for (int k = 0; k < m; ++k) {
      if (mixed) {
        launch_apply_batch<float>(P.hc, P.totG, cs, P.a32, P.amap, true);
        k_update_batch<float><<<P.totG2, BLOCK, 0, cs>>>(P.u32, P.umap);
      } else {
        launch_apply_batch<double>(P.hc, P.totG, cs, P.af64, P.amap, true);
        k_update_batch<double><<<P.totG2, BLOCK, 0, cs>>>(P.u64, P.umap);
      }
    }
    if (mixed) {
      k_b_formw<<<P.totG2, BLOCK, 0, cs>>>(P.be, P.umap, 1);
      launch_apply_batch<double>(P.hc, P.totG, cs, P.a64, P.amap, false);
      k_b_resid<<<P.totG2, BLOCK, 0, cs>>>(P.be, P.umap, 1);
      k_b_fin<<<nvar, BLOCK, 0, cs>>>(P.be, 1, 0, rtol2, P.flags);
    } else {
      k_b_flags<<<(nvar + 255) / 256, 256, 0, cs>>>(P.be, nvar, P.flags);
    }
    he = hipStreamEndCapture(cs, &graph);
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    set_error("graph capture: %s", hipGetErrorString(he));
    status = MFP_E_HIP;
  }
  std::vector<int> hflags(nvar, 0);
  long long launches = 0;
  const long long max_launches = (opts->kmax + m - 1) / m + 1;
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
    // true residual of every system
    k_b_formw<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, 0);
    launch_apply_batch<double>(P.hc, P.totG, st, P.a64, P.amap, false);
    k_b_resid<<<P.totG2, BLOCK, 0, st>>>(P.be, P.umap, 2);
    k_b_fin<<<nvar, BLOCK, 0, st>>>(P.be, 2, 0, rtol2, P.flags);
    MFP_TRY_HIP(hipGetLastError());
  }
  // outputs
  std::vector<DevState> hs(nvar), hin(nvar);
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
    if (mixed)
      MFP_TRY_HIP(hipMemcpyAsync(&hin[i], w.st2, sizeof(DevState), hipMemcpyDeviceToHost, st));
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
    const long long it = s.iters;
    const double* xb = s.xb[it & 1];
    for (int b = 0; b < nb; ++b) psi_b_h[(size_t)i * nb + b] = xb[b];
    if (copfi_h && pair_lo >= 0 && pair_hi >= 0) {
      const mfp_circle* ci = circles_h + (size_t)i * nb;
      copfi_h[i] = (xb[pair_hi] - xb[pair_lo]) / (flow->U * (ci[pair_hi].cy - ci[pair_lo].cy));
    }
    const int code = mixed ? s.done : s.done;
    if (code == 2) worst = MFP_E_BREAKDOWN;
    if ((code == 3 || code == 0) && worst == MFP_OK) worst = MFP_W_NOCONV;
    if (stats_h) {
      mfp_stats& o = stats_h[i];
      std::memset(&o, 0, sizeof(o));
      o.iters = it;
      o.outer_iters = mixed ? s.outer_count : 0;
      o.applies = it + (mixed ? s.outer_count + 1 : 2);
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
