// One conjugate-gradient iteration per kernel launch.
//
// The paper's Algorithm 1 runs the textbook CG loop: apply the operator to the
// direction, alpha, update of the iterate and the residual, beta, new direction.  Done
// as written that needs two grid-wide reductions per iteration (p.Ap before alpha,
// r.r before beta), i.e. two kernels.  Here launch j does both halves for iteration j
// with the same recurrences:
//
//   alpha_{j-1} = |r_{j-1}|^2 / p_{j-1}.Kp_{j-1}           (partials of launch j-1)
//   x_j = x_{j-1} + alpha p_{j-1},   r_j = r_{j-1} - alpha Kp_{j-1}
//   |r_j|^2 = |r_{j-1}|^2 - 2 alpha r_{j-1}.Kp_{j-1} + alpha^2 Kp_{j-1}.Kp_{j-1}
//   beta_j = |r_j|^2 / |r_{j-1}|^2,  p_j = r_j + beta_j p_{j-1},  Kp_j
//
// with per-block partials of r_j.r_j, p_j.Kp_j, r_j.Kp_j and Kp_j.Kp_j for launch j+1.
// Only |r_j|^2 inside beta_j (and the stopping test) comes from the expansion, over the
// free nodes; alpha always uses the sum of the squares of the stored residual of the
// previous launch, so the expansion's rounding never accumulates.  Body unknowns
// (one per body, the multi-point constraint rows) follow the same recurrences as
// scalars, their K p entries being the per-body sums of K p over the body's nodes.
//
// Every block needs r_j, p_j at the halo of its tasks, so it recomputes them there
// from r_{j-1}, Kp_{j-1}, p_{j-1} (the same arithmetic as the owner); r, p and Kp are
// therefore double-buffered by parity (launch j reads slot (j-1)&1 and writes j&1),
// as are the partials and the per-body slot sums.  The iterate is read and written
// at owned nodes only, and only by odd launches, two directions at a time:
// x_j = x_{j-2} + alpha_{j-2} p_{j-2} + alpha_{j-1} p_{j-1} (p_{j-2} is still in the
// slot launch j overwrites; each owner reads it before writing p_j), which saves one
// store stream in two launches.
//
// Launch k0 starts (or restarts) a run: alpha = 0, |r_j|^2 is the exact sum of the
// start residual (partials written by k_step_start), beta_j = |r_j|^2 / rr_prev with
// rr_prev = 0 for a fresh start (direction p_{j-1} = 0) or, after a residual
// replacement, the exact |r_{j-1}|^2 kept by the launch that stopped.
//
// A launch that finds |r_j|^2 <= the threshold, j >= kmax, a breakdown or a non-finite
// value records the outcome (iterate index j, alpha) and returns; k_finish then adds
// the directions the iterate still lacks.
#pragma once

#include "apply.h"

namespace mfp {

// Global memory.  The iteration kernel accesses its vectors through pointers of this
// address space: pointers that a kernel loads from memory (the batched argument
// tables) are otherwise generic, and every access through them becomes a flat
// instruction (which also waits on the LDS counter).
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* as_global(T* p) {
  return (gmem<T>*)p;
}

// Element at a 32-bit byte offset from a uniform base pointer (lets the compiler use
// scalar-base + 32-bit vector-offset addressing; the solver's vectors are < 4 GiB).
template <typename T>
__device__ __forceinline__ T ld_at(const gmem<T>* base, unsigned boff) {
  return *reinterpret_cast<const gmem<T>*>(reinterpret_cast<const gmem<char>*>(base) + boff);
}
// Store of the iteration's vectors; STREAM: not kept in L2 (non-temporal).  For
// working sets larger than the memory-side cache the streaming form measured ~11%
// faster per iteration (the stores no longer evict the halo rows that neighbouring
// tasks re-read); for smaller ones the cached form is faster (the next iteration
// finds the data in cache).  A compile-time choice: with a run-time branch the
// compiler merges the two stores and drops the hint.
template <bool STREAM, typename T>
__device__ __forceinline__ void st_vec(gmem<T>* base, unsigned boff, T v) {
  gmem<T>* p = reinterpret_cast<gmem<T>*>(reinterpret_cast<gmem<char>*>(base) + boff);
  if constexpr (STREAM)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <typename T>
struct StepArgs {
  int P, nstrip, nchunk;         // pitch, strips, chunks (task t = chunk * nstrip + strip)
  const uint8_t* tplain;         // per task, 1: constant-stencil task
  const int8_t* tag;
  const T* dx;                   // displacement / hx
  const T* dy;
  const unsigned long long* tbody;
  const int* tslot;
  int nslots;                    // body-sum slots in use
  // vectors of iteration j-1 (parity slot (j-1)&1) and j (slot j&1), chosen by the
  // host for every launch so that no address depends on a loaded value
  const T* rp;                   // residual
  const T* qp;                   // K p
  const T* pp;                   // direction
  T* rc;
  T* qc;
  T* pc;
  T* x;                          // iterate (free nodes meaningful)
  const double* part_p;          // per-block partials: r.r, p.Kp, r.Kp, Kp.Kp
  double* part_c;
  const double* bpart_p;         // per-slot, per-body sums of K p
  double* bpart_c;
  DevState* st;
  int nb;
  int npart0;                    // partials (blocks) written by the start kernel
  int stream;                    // 1: launch the streaming-store instance
  long long k0;                  // start launch of this run
  long long j;                   // this launch
  T cC, cE, cN, cD;              // constant stencil
  T ry;                          // hy / hx
  // batched launches (k_step_batch): the launch index is st->jbase + the launch's offset
  // in the replayed block and the start launch is st->k0; the parity slots below
  // replace the per-launch pointers; G = this system's blocks
  int G;
  int* host_done;                // single solve: stop code also written here (pinned host)
  double* hist;                  // single solve, may be NULL: hist[2j] = alpha_{j-1} and
  long long hist_cap;            // hist[2j+1] = beta_j as launch j forms them (j < hist_cap)
  const T* kcoef;                // stored element entries (KST instances): slab per task
  const int* tgeo;               // per task: its slab, -1 for constant-stencil tasks
  const int2* wtask;             // 8-wavefront blocks: one task per wavefront, entry
                                 // blockIdx * 8 + wave = (task or -1, flags: bit 0 constant
                                 // stencil, bit 1 body nodes, bits 2..15 body-sum slot + 1,
                                 // bits 16..30 stored-entry slab + 1)
  T* rs[2];
  T* ps[2];
  T* qs[2];
  double* parts[2];
  double* bparts[2];
};

// Work distribution: the launch keeps all its wavefronts resident; wavefront w takes
// tasks w, w + W, w + 2W, ... (W wavefronts, tasks in strip-fastest order), so that at
// any time the wavefronts of the chip cover a few contiguous bands of rows and each
// XCD one contiguous part of every band (its L2 serves the halo rows and columns that
// neighbouring tasks share).  Every task's rows, iterate rows and flags are requested
// one task ahead (a task that evaluates geometry requests its tags and displacements
// first and the next task's data after its cell march, which needs the registers).
// BATCH: a launch of k_step_batch (launch index and parity slots from the device
// state).  A compile-time choice: with a run-time branch there the compiler splits the
// kernel-argument loads into several dependent round trips ahead of the first vector
// load.
template <typename T, int HC, bool STREAM, bool XUPD, bool KST, int NW = WAVES, bool BATCH = false>
__device__ __forceinline__ void step_core(const StepArgs<T>& a, const int vblk, const int G,
                                          const int koff, double* s_red, double* s_pb,
                                          double* s_qb) {
  constexpr int NT = NW * 64;  // threads per block
  // 8-wavefront blocks take their one task and its flags from a table (a.wtask)
  constexpr bool TAB = NW == 8;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  // consecutive virtual blocks share an XCD (work-groups are dealt round-robin to 8 XCDs;
  // vblk and blockIdx.x agree modulo 8)
  const int vb = (vblk & 7) * (G >> 3) + (vblk >> 3);
  const unsigned P = (unsigned)a.P;
  const int nstrip = a.nstrip;
  const int ntask = nstrip * a.nchunk;
  const bool owner = lane >= 1 && lane <= SW;
  const int W = G * NW;
  long long j = a.j, k0 = a.k0;
  gmem<DevState>* const st = as_global(a.st);
  const T* rp = a.rp;
  const T* qp = a.qp;
  const T* pp = a.pp;
  T* rc = a.rc;
  T* qc = a.qc;
  T* pc = a.pc;
  const double* part_p = a.part_p;
  double* part_c = a.part_c;
  const double* bpart_p = a.bpart_p;
  double* bpart_c = a.bpart_c;
  if constexpr (BATCH) {
    // The launch index must arrive before any vector is requested (the parity slots
    // depend on it), so the stop flag comes with it and a stopped system's blocks
    // leave before they request anything.  One thread reads, the block decides
    // together (see the stop decision below).
    long long* const s_hdr = reinterpret_cast<long long*>(s_red + 4 * NW + 1);
    if (tid == 0) {
      s_hdr[0] = st->jbase;
      s_hdr[1] = st->k0;
      s_hdr[2] = st->done;
    }
    __syncthreads();
    if (s_hdr[2] != 0) return;
    j = s_hdr[0] + koff;
    k0 = s_hdr[1];
    const bool c = (j & 1) != 0;  // selects, not indexing (keeps the table in registers)
    rp = c ? a.rs[0] : a.rs[1];
    qp = c ? a.qs[0] : a.qs[1];
    pp = c ? a.ps[0] : a.ps[1];
    rc = c ? a.rs[1] : a.rs[0];
    qc = c ? a.qs[1] : a.qs[0];
    pc = c ? a.ps[1] : a.ps[0];
    part_p = c ? a.parts[0] : a.parts[1];
    part_c = c ? a.parts[1] : a.parts[0];
    bpart_p = c ? a.bparts[0] : a.bparts[1];
    bpart_c = c ? a.bparts[1] : a.bparts[0];
  }
  const gmem<T>* const rpg = as_global(rp);
  const gmem<T>* const qpg = as_global(qp);
  const gmem<T>* const ppg = as_global(pp);
  gmem<T>* const rcg = as_global(rc);
  gmem<T>* const qcg = as_global(qc);
  gmem<T>* const pcg = as_global(pc);
  const gmem<double>* const part_pg = as_global(part_p);
  gmem<double>* const part_cg = as_global(part_c);
  const gmem<double>* const bpart_pg = as_global(bpart_p);
  gmem<double>* const bpart_cg = as_global(bpart_c);
  gmem<T>* const xg = as_global(a.x);
  const gmem<uint8_t>* const tplain = as_global(a.tplain);
  const gmem<unsigned long long>* const tbody = as_global(a.tbody);
  const gmem<int>* const tslot = as_global(a.tslot);
  const gmem<int8_t>* const tagg = as_global(a.tag);
  const gmem<T>* const dxg = as_global(a.dx);
  const gmem<T>* const dyg = as_global(a.dy);
  const int cur = (int)(j & 1), prv = cur ^ 1;
  const bool start = j == k0;
  constexpr unsigned TS = sizeof(T);
  const unsigned RB = P * TS;  // bytes per padded row of a T vector
  // task t: rows 0..HC+1 are padded rows chunk*HC + r, lane is column strip*64 + lane
  // (it reads column strip*64 + lane + halo_shift)
  auto node0 = [&](int t) -> unsigned {
    const int m = t % nstrip, kc = t / nstrip;
    return (unsigned)(kc * HC) * P + (unsigned)(m * 64 + lane);
  };
  auto shift_of = [&](int t) -> int { return halo_shift(lane, t % nstrip, nstrip); };

  // next task's data (requested one task ahead)
  T nr[HC + 2], nq[HC + 2], np[HC + 2], nx[HC], n2[HC];  // n2: p_{j-2} (XUPD)
  int n_plain = 1, n_body = 0, n_slot = -1, n_geo = 0;
  // Wavefront u takes tasks u, u + W, u + 2W, ... through the full rounds (F = ntask / W
  // of them).  The last, partial round's R tasks go out in eight contiguous runs, one to
  // each XCD's group of W / 8 wavefronts (u / (W / 8) is the XCD): dealt to the first R
  // wavefronts, as a full round is, they would all sit on the first XCDs, which would
  // then run that round alone while the rest of the chip waited for the launch's end
  // (2048x1024, 8738 tasks over 2048 wavefronts: the last 7-11 us of a 24-33 us launch).
  const int u = vb * NW + wv;
  const int F = ntask / W, FW = F * W, R = ntask - FW;
  const int gw = W >> 3, gx = u / gw, gl = u - gx * gw;
  const int rb = (gx * R) >> 3, re = ((gx + 1) * R) >> 3;
  const int t_last = gl < re - rb ? FW + rb + gl : ntask;  // its task of the last round
  int t = F > 0 ? u : t_last, tflags = 1;  // first task, table flags
  const gmem<int>* const tgeo = as_global(a.tgeo);
  auto fetch = [&](int t) {
    if constexpr (TAB) {
      n_plain = tflags & 1;
      n_body = (tflags >> 1) & 1;
      n_slot = ((tflags >> 2) & 0x3fff) - 1;
      if (KST) n_geo = ((tflags >> 16) & 0x7fff) - 1;
    } else {
      // flags first: the geometry request waits for them, not for the rows
      n_plain = tplain[t];
      n_body = tbody[t] != 0ull;
      n_slot = tslot[t];
      if (KST) n_geo = tgeo[t];
    }
    const unsigned bo = (unsigned)((int)node0(t) + shift_of(t)) * TS;
#pragma unroll
    for (int r = 0; r < HC + 2; ++r) {
      nr[r] = ld_at(rpg, bo + r * RB);
      nq[r] = ld_at(qpg, bo + r * RB);
      np[r] = ld_at(ppg, bo + r * RB);
    }
    if (XUPD) {
      // own rows only (halo lanes' values are unused)
#pragma unroll
      for (int r = 0; r < HC; ++r) {
        nx[r] = ld_at(xg, bo + (r + 1) * RB);
        n2[r] = ld_at((const gmem<T>*)pcg, bo + (r + 1) * RB);
      }
    }
  };
  // ---- scalars of iteration j ----
  // Everything they need is requested first, in one round trip, ahead of the task's
  // rows: the previous launch's partials, the state, lane b's body values and the
  // per-body slot sums (wave w: bodies w and w + 4 from the first 64 slots; more
  // bodies or slots in a second pass).  These loads, and the rows', are unconditional
  // (clamped indices, values past the end dropped when used): the counter a wavefront
  // waits on counts loads in issue order, and a load under a branch makes the wait for
  // anything issued before it a wait for everything.  So the scalars are reduced while
  // the rows travel, and the first task's geometry is requested right after the flags
  // arrive, together with the partials.
  // The scalar phase (inputs in, wavefront sums, the block barrier, alpha and beta) runs
  // at raised wave priority: the SIMD's other wavefront, already in its task, yields to
  // it, so the block reaches its barrier sooner (1024x512: 13.73 -> 13.29 us per launch;
  // 4096x2048 unchanged).  Back to normal priority for the task.
  __builtin_amdgcn_s_setprio(3);
  const int npart = start ? a.npart0 : G;  // at least 1
  const gmem<double>* const pt = part_pg;
  constexpr int PU = 2;
  double pv[PU][4];
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const int i = min(tid + u * NT, npart - 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) pv[u][c] = pt[4 * i + c];
  }
  const int nb = a.nb, nsl = a.nslots;
  const int done = st->done;
  const double rr_stop = st->rr_stop, rr_prev_start = st->rr_prev, stop_rel = st->stop_rel;
  const double alpha2 = st->alpha_hist[prv];  // alpha_{j-2}
  const long long kmax = st->kmax;
  // lane b: body b of iteration j-1 (the state holds MFP_MAX_BODIES = 64 of each)
  const bool lb = lane < nb;
  const double rbp_l = st->rb[prv][lane], pbp_l = st->pb[prv][lane], xbp_l = st->xb[prv][lane];
  // slot sums of bodies b0, b1 (K p of iteration j-1); the slot buffer holds at least
  // 64 slots of max(nb, 1) bodies
  const gmem<double>* const bq = bpart_pg;
  const int b0 = wv, b1 = wv + NW;
  const int nbc = nb > 0 ? nb : 1;
  const double q0_l = bq[(long long)lane * nb + min(b0, nbc - 1)];
  const double q1_l = bq[(long long)lane * nb + min(b1, nbc - 1)];
  if constexpr (TAB) {
    // the table's entry: the wavefront's task and its flags, by a scalar load issued
    // behind the vector loads above (which then travel while it waits).  Written out:
    // the compiler issues a table load that it cannot prove unwritten as a vector load,
    // and waiting for that one would wait for every vector load before it; and a scalar
    // load it places first delays those vector loads by its round trip.  The asm waits
    // for its own result.
    __builtin_amdgcn_sched_barrier(0);
    const long long* const ep =
        reinterpret_cast<const long long*>(a.wtask) + vblk * NW + __builtin_amdgcn_readfirstlane(wv);
    long long e;
    asm volatile("s_load_dwordx2 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(e) : "s"(ep));
    const int ex = (int)(unsigned)e;  // int2 (x, y) in memory: x in the low word
    t = ex >= 0 ? ex : ntask;
    tflags = (int)(e >> 32);
  }
  fetch(t < ntask ? t : ntask - 1);  // a wavefront without a task drops what it fetched

  int8_t tg[HC + 2];
  T ddx[HC + 2], ddy[HC + 2];
  T kc[HC + 1][KCOEF];  // KST: the task's stored element entries
  const gmem<T>* const kcg = as_global(a.kcoef);
  // tags, and either the displacements (geometry on the fly) or the element entries
  auto load_geom = [&](int tt, int slab) {
    const unsigned ln0 = (unsigned)((int)node0(tt) + shift_of(tt));
#pragma unroll
    for (int r = 0; r < HC + 2; ++r) tg[r] = ld_at(tagg, ln0 + r * P);
    if constexpr (KST) {
      const unsigned kb = ((unsigned)slab * (unsigned)kslab<HC>() + (unsigned)lane) * TS;
#pragma unroll
      for (int r = 0; r <= HC; ++r)
#pragma unroll
        for (int e = 0; e < KCOEF; ++e) kc[r][e] = ld_at(kcg, kb + (r * KCOEF + e) * 64 * TS);
    } else {
#pragma unroll
      for (int r = 0; r < HC + 2; ++r) {
        ddx[r] = ld_at(dxg, ln0 * TS + r * RB);
        ddy[r] = ld_at(dyg, ln0 * TS + r * RB);
      }
    }
  };
  // with the table the flags came with the task: the geometry follows the rows at once
  // (stored entries, 36 or 72 registers, wait for the task: held through the scalar
  // phase, they made the FP64 kernel spill)
  if constexpr (TAB && !KST) {
    if (t < ntask && !n_plain) load_geom(t, n_geo);
  }
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const bool in = tid + u * NT < npart;
    s0 += in ? pv[u][0] : 0.0;
    s1 += in ? pv[u][1] : 0.0;
    s2 += in ? pv[u][2] : 0.0;
    s3 += in ? pv[u][3] : 0.0;
  }
  if constexpr (!TAB) {
    if (t < ntask && !n_plain) load_geom(t, n_geo);
  }
  for (int i = tid + PU * NT; i < npart; i += NT) {  // launches of more than 512 blocks
    s0 += pt[4 * i];
    s1 += pt[4 * i + 1];
    s2 += pt[4 * i + 2];
    s3 += pt[4 * i + 3];
  }
  const double rbp = lb ? rbp_l : 0.0, pbp = lb ? pbp_l : 0.0, xbp = lb ? xbp_l : 0.0;
  const bool qin = !start && lane < nsl;
  double q0 = qin && b0 < nb ? q0_l : 0.0;
  double q1 = qin && b1 < nb ? q1_l : 0.0;
  if (!start) {
    for (int sl = lane + 64; sl < nsl; sl += 64) {
      if (b0 < nb) q0 += bq[(long long)sl * nb + b0];
      if (b1 < nb) q1 += bq[(long long)sl * nb + b1];
    }
  }
  // wave sums, six independent chains.  A wavefront skips the chains whose lanes are
  // all zero: the partials when the previous launch had no more blocks than the
  // wavefronts before it have lanes (a table launch of 256 blocks: wavefronts 4..7),
  // the slot sums of bodies that do not exist.  All of a block's wavefronts run this
  // FP64 arithmetic at once, two to a SIMD, so the idle chains cost the others issue
  // slots.
  if (npart > wv * 64) {
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
  }
  if (b0 < nb) q0 = wave_sum(q0);
  if (b1 < nb) q1 = wave_sum(q1);
  if (lane == 0) {
    s_red[4 * wv] = s0;
    s_red[4 * wv + 1] = s1;
    s_red[4 * wv + 2] = s2;
    s_red[4 * wv + 3] = s3;
    if (b0 < nb) s_qb[b0] = start ? 0.0 : q0;
    if (b1 < nb) s_qb[b1] = start ? 0.0 : q1;
    // the block leaves on wave 0's reading of the stop flag: the waves read it at
    // different times, and block 0 may set it during this launch (a wave that left
    // alone would leave its share of the block sums unwritten)
    if (wv == 0) s_red[4 * NW] = done ? 1.0 : 0.0;
  }
  // bodies beyond 2 NW (rare)
  for (int b = wv + 2 * NW; b < nb; b += NW) {
    double v = 0.0;
    if (!start)
      for (int sl = lane; sl < nsl; sl += 64) v += bq[(long long)sl * nb + b];
    v = wave_sum(v);
    if (lane == 0) s_qb[b] = v;
  }
  __syncthreads();
  if (s_red[4 * NW] != 0.0) return;  // stopped (the same decision in every wave)
  const double qb = lane < nb ? s_qb[lane] : 0.0;
  // body parts of r.r and p.Kp, two independent chains
  const double brr = wave_sum(rbp * rbp), bpq = wave_sum(pbp * qb);
  const double S_rr = wave_tree<NW>(s_red);
  const double S_pq = wave_tree<NW>(s_red + 1);
  const double S_rq = wave_tree<NW>(s_red + 2);
  const double S_qq = wave_tree<NW>(s_red + 3);
  double alpha = 0.0, rr_prev;
  int code = 0;
  if (start) {
    rr_prev = rr_prev_start;
  } else {
    rr_prev = S_rr + brr;
    const double pq = S_pq + bpq;
    if (!(pq > 0.0) || !isfinite(pq)) code = 2;
    alpha = code ? 0.0 : rr_prev / pq;
  }
  const double rbj = rbp - alpha * qb;
  const double xbj = xbp + alpha * pbp;
  // the body part of |r_j|^2 is summed exactly: a body residual can drop by orders
  // of magnitude in one iteration, where the expansion would cancel
  const double b_rr = wave_sum(rbj * rbj);
  const double rr_j =
      start ? S_rr + b_rr : (S_rr - 2.0 * alpha * S_rq + alpha * alpha * S_qq) + b_rr;
  const double stop = (start && stop_rel > 0.0) ? stop_rel * rr_j : rr_stop;
  if (!code) {
    if (!isfinite(rr_j))
      code = 2;
    else if (rr_j <= stop)
      code = 1;
    else if (j >= kmax)
      code = 3;
  }
  const double beta = rr_prev > 0.0 ? rr_j / rr_prev : 0.0;
  const double pbj = rbj + beta * pbp;
  if (vblk == 0 && wv == 0) {
    if (lane < nb) {
      st->rb[cur][lane] = rbj;
      st->xb[cur][lane] = xbj;
      if (!code) st->pb[cur][lane] = pbj;
    }
    if (lane == 0) {
      // the CG scalars, for the Lanczos condition estimate (a restart launch has no
      // step length, a stopping one forms no direction)
      if (a.hist && j < a.hist_cap) {
        if (!start) a.hist[2 * j] = alpha;
        if (!code) a.hist[2 * j + 1] = beta;
      }
      st->alpha = alpha;
      st->alpha_hist[cur] = alpha;
      st->rr[cur] = rr_j;
      if (start && stop_rel > 0.0) st->rr_stop = stop;
      if (code) {
        st->done = code;
        st->iters = j;
        st->rr_final = rr_j;
        st->rr_prev = rr_prev;
        if (a.host_done) *a.host_done = code;  // pinned host memory the host polls
      } else {
        st->beta = beta;
      }
    }
  }
  if (code) return;
  if constexpr (!TAB) {
    if (wv == 0 && lane < nb) s_pb[lane] = pbj;
    __syncthreads();
  }
  // the table launch needs no second barrier: every wavefront holds the same body
  // values (lane b: body b) and its tasks read them from its own lanes
  const T al = (T)alpha, be = (T)beta, al2 = (T)alpha2;
  __builtin_amdgcn_s_setprio(0);

  // ---- tasks ----
  double prr = 0.0, ppq = 0.0, prq = 0.0, pqq = 0.0;
  bool first = true;
  // one task: its rows are in nr, nq, np (and nx, n2); next() requests the next task's
  auto task = [&](const int t, const bool plain, const bool bm, const int slot, const int geo,
                  auto&& next) {
    const unsigned n0 = node0(t);
    const unsigned bo = n0 * TS;
    // r_j, p_j (as at a free node until corrected) and p_{j-1} at rows 0..HC+1
    // and the new iterate at the owned rows (odd launches), formed at once so that the
    // old directions and iterate need no registers during the cell march
    T rj[HC + 2], v[HC + 2], xn[HC];
#pragma unroll
    for (int r = 0; r < HC + 2; ++r) {
      rj[r] = nr[r] - al * nq[r];
      v[r] = rj[r] + be * np[r];
    }
    if (XUPD) {
#pragma unroll
      for (int r = 0; r < HC; ++r) xn[r] = (nx[r] + al2 * n2[r]) + al * np[r + 1];
    }
    if (!plain && (!first || (TAB && KST))) load_geom(t, geo);
    first = false;
    T qr[HC];
    if (plain) {
      next();
      stencil_task<T, HC>(a.cC, a.cE, a.cN, a.cD, v, qr);
    } else {
      // body nodes carry p_b, Dirichlet and halo nodes 0 (r is zero there); the
      // potential's body nodes (negative tags) keep their own p
#pragma unroll
      for (int r = 0; r < HC + 2; ++r) {
        const int8_t g = tg[r];
        if constexpr (TAB) {
          // every lane takes part in the lane permute; lanes off a body read their own
          const double pv = __shfl(pbj, g >= TAG_BODY0 ? g - TAG_BODY0 : lane);
          if (g >= TAG_BODY0)
            v[r] = (T)pv;
          else if (g > TAG_FREE)
            v[r] = (T)0;
        } else {
          if (g >= TAG_BODY0)
            v[r] = (T)s_pb[g - TAG_BODY0];
          else if (g > TAG_FREE)
            v[r] = (T)0;
        }
      }
      if constexpr (KST)
        march_task_stored<T, HC>(v, kc, qr);
      else
        march_task<T, HC>(a.ry, lane, tg, v, ddx, ddy, qr);
      // requested after the cell march, which needs the registers
      next();
    }
    double bacc = 0.0;
#pragma unroll
    for (int r = 1; r <= HC; ++r) {
      const unsigned go = bo + r * RB;
      const int8_t g = plain ? (int8_t)TAG_FREE : tg[r];
      const bool fr = tag_own(g);  // free (the potential's body nodes too)
      const T qv = (owner && fr) ? qr[r - 1] : (T)0;
      // every lane stores (the padding lanes zeros): whole aligned rows
      st_vec<STREAM>(rcg, go, owner ? rj[r] : (T)0);
      st_vec<STREAM>(pcg, go, owner ? v[r] : (T)0);
      st_vec<STREAM>(qcg, go, qv);
      if (XUPD) st_vec<STREAM>(xg, go, owner ? xn[r - 1] : (T)0);
      if (owner) {
        if (fr) {
          const double rd = (double)rj[r], qd = (double)qv;
          prr += rd * rd;
          ppq += (double)v[r] * qd;
          prq += rd * qd;
          pqq += qd * qd;
        }
      }
      if (bm) body_row(owner, g, (double)qr[r - 1], lane, bacc);
    }
    if (bm && lane < nb) bpart_cg[(long long)slot * nb + lane] = bacc;
  };
  if constexpr (TAB) {
    // one task, nothing to request after it
    if (t < ntask) task(t, n_plain != 0, n_plain == 0 && n_body != 0, n_slot, n_geo, [] {});
  } else {
    while (t < ntask) {
      const bool plain = n_plain != 0;
      const int tn = t + W < FW ? t + W : (t < FW ? t_last : ntask);
      task(t, plain, !plain && n_body != 0, n_slot, n_geo, [&] {
        if (tn < ntask) fetch(tn);
      });
      t = tn;
    }
  }
  // four block sums, fixed order
  prr = wave_sum(prr);
  ppq = wave_sum(ppq);
  prq = wave_sum(prq);
  pqq = wave_sum(pqq);
  // into LDS that nothing reads before this point (s_red is still being read by waves
  // that have not finished their scalars), so one barrier suffices
  double* const s_fin = s_qb + MFP_MAX_BODIES;
  if (lane == 0) {
    s_fin[4 * wv] = prr;
    s_fin[4 * wv + 1] = ppq;
    s_fin[4 * wv + 2] = prq;
    s_fin[4 * wv + 3] = pqq;
  }
  __syncthreads();
  if (tid < 4) {
    part_cg[4 * vblk + tid] = wave_tree<NW>(s_fin + tid);
  }
}

// NW wavefronts per block: 4, or 8 for launches with one task per wavefront from a
// table (one block per CU; wavefronts w and w + 4 of a block share a SIMD).
template <typename T, int HC, bool STREAM, bool XUPD, bool KST, int NW = WAVES>
__global__ void __launch_bounds__(NW * 64) k_step(StepArgs<T> a) {
  __shared__ double s_red[4 * NW + 4];  // + stop flag, launch header (batched)
  __shared__ double s_pb[MFP_MAX_BODIES];
  __shared__ double s_qb[MFP_MAX_BODIES + 4 * NW];  // + final block sums
  step_core<T, HC, STREAM, XUPD, KST, NW>(a, blockIdx.x, gridDim.x, 0, s_red, s_pb, s_qb);
}

// Many independent systems in one launch: block b works for system map[b].x as its
// virtual block map[b].y (each system's blocks start at a multiple of 8); koff is this
// launch's offset in the replayed block of launches; tasks of HC node rows (the
// layouts').
template <typename T, int HC, bool XUPD, bool KST>
__global__ void __launch_bounds__(BLOCK) k_step_batch(const StepArgs<T>* __restrict__ args,
                                                      const int2* __restrict__ map, int koff) {
  __shared__ double s_red[4 * WAVES + 4];  // + stop flag, launch header
  __shared__ double s_pb[MFP_MAX_BODIES];
  __shared__ double s_qb[MFP_MAX_BODIES + 4 * WAVES];  // + final block sums
  const int2 vm = map[blockIdx.x];
  const StepArgs<T>& a = args[vm.x];
  // streaming stores: the systems' vectors together exceed the memory-side cache
  // (measured on a 256-system sweep: 2% faster than cached stores)
  step_core<T, HC, true, XUPD, KST, WAVES, true>(a, vm.y, a.G, koff, s_red, s_pb, s_qb);
}

// Tasks of HC node rows (the layout's); odd launches update the iterate; a.stream
// selects the streaming-store instance, a.kcoef the stored-element-entry one.
template <typename T, int HC, bool KST>
inline void launch_step_k(int G, hipStream_t st, const StepArgs<T>& a) {
  const bool xu = (a.j & 1) != 0;
  if (a.wtask) {
    // one task per wavefront from the table: G blocks of 8 wavefronts, one per CU
    constexpr int T8 = 8 * 64;
    if (a.stream) {
      if (xu)
        k_step<T, HC, true, true, KST, 8><<<G, T8, 0, st>>>(a);
      else
        k_step<T, HC, true, false, KST, 8><<<G, T8, 0, st>>>(a);
    } else {
      if (xu)
        k_step<T, HC, false, true, KST, 8><<<G, T8, 0, st>>>(a);
      else
        k_step<T, HC, false, false, KST, 8><<<G, T8, 0, st>>>(a);
    }
    return;
  }
  if (a.stream) {
    if (xu)
      k_step<T, HC, true, true, KST><<<G, BLOCK, 0, st>>>(a);
    else
      k_step<T, HC, true, false, KST><<<G, BLOCK, 0, st>>>(a);
  } else {
    if (xu)
      k_step<T, HC, false, true, KST><<<G, BLOCK, 0, st>>>(a);
    else
      k_step<T, HC, false, false, KST><<<G, BLOCK, 0, st>>>(a);
  }
}

template <typename T, int HC>
inline void launch_step_h(int G, hipStream_t st, const StepArgs<T>& a) {
  if (a.kcoef)
    launch_step_k<T, HC, true>(G, st, a);
  else
    launch_step_k<T, HC, false>(G, st, a);
}

// hc: the layout's task height: 4; 5 for FP64 where 4-row tasks would outnumber the
// resident wavefronts and 5-row ones do not; 8 for large FP32 layouts (FP32 8-row
// tasks use about as many registers as FP64 4-row ones; FP64 8-row tasks would need
// 256 and run one wavefront per SIMD).
template <typename T>
inline void launch_step(int G, hipStream_t st, const StepArgs<T>& a, int hc) {
  if (hc == 8)
    launch_step_h<T, 8>(G, st, a);
  else if (hc == 5)
    launch_step_h<T, 5>(G, st, a);
  else
    launch_step_h<T, 4>(G, st, a);
}

// Start (or restart after a residual replacement) of a run at launch k0: the
// residual slot (k0-1)&1 takes r (converted from the FP64 residual when they
// differ), and its per-block partials are (r.r, 0, 0, 0) in the step layout.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_step_start(long long n, const double* __restrict__ r64,
                                                      T* __restrict__ rdst,
                                                      double* __restrict__ part) {
  __shared__ double s_red[BLOCK / 64];
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const T v = (T)r64[e];
    if ((const void*)rdst != (const void*)r64) rdst[e] = v;
    acc += (double)v * (double)v;
  }
  const double bs = block_sum(acc, s_red);
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = threadIdx.x == 0 ? bs : 0.0;
}

// Single block: body state of slot `slot` for a run start.  rb = the FP64 body
// residuals of the outer state (slot 0), xb = 0 when the iterate is a correction
// (inner solve) or kept otherwise; p_b = 0 and rr_prev = 0 for a fresh start, kept
// for a restart; stop_rel > 0 sets the threshold relative to the start residual.
__global__ void k_step_bodies(const DevState* outer, DevState* in, int nb, int slot,
                              int fresh, int correction, double stop_rel, long long kmax) {
  const int b = threadIdx.x;
  if (b < nb) {
    in->rb[slot][b] = outer->rb[0][b];
    if (correction) in->xb[slot][b] = 0.0;
    else if (in != outer) in->xb[slot][b] = outer->xb[0][b];
    if (fresh) in->pb[slot][b] = 0.0;
  }
  if (b == 0) {
    // no direction is pending in the iterate at a start
    in->alpha_hist[0] = 0.0;
    in->alpha_hist[1] = 0.0;
    if (fresh) in->rr_prev = 0.0;
    in->stop_rel = stop_rel;
    in->kmax = kmax;
    in->done = 0;
  }
}

// The iterate after the launch J that stopped: x_J = x_{J-1} + alpha_{J-1} p_{J-1}.
// If launch J-1 was odd, x holds x_{J-1}; otherwise it holds x_{J-2} and also lacks
// alpha_{J-2} p_{J-2} (p_{J-2} is still in slot J&1: launch J wrote no direction).
template <typename T>
__global__ void k_finish(long long n, T* __restrict__ x, const T* __restrict__ p0,
                         const T* __restrict__ p1, const DevState* __restrict__ st) {
  const long long J = st->iters;
  const T a1 = (T)st->alpha;
  const bool two = ((J - 1) & 1) == 0;
  const T a2 = two ? (T)st->alpha_hist[(J - 1) & 1] : (T)0;
  const T* pa = ((J - 1) & 1) ? p1 : p0;  // p_{J-1}
  const T* pb = (J & 1) ? p1 : p0;        // p_{J-2}
  if (a1 == (T)0 && a2 == (T)0) return;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    x[e] = (x[e] + a2 * pb[e]) + a1 * pa[e];
}

}  // namespace mfp
