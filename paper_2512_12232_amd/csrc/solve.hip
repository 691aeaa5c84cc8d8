// Constrained stream-function solve: setup, conjugate-gradient kernels and the
// host drivers of mfp_psi_solve, mfp_phi_solve (the velocity potential: body nodes
// as unknowns of their own, see the tags in mfp_internal.h) and mfp_element_apply.
//
// Unknowns (section "Matrix-Free Conjugate Gradient with Multiple Constraint
// Enforcement"): free nodes plus one value psi_b per body, N_dof = N_int + N_N + N_b.
// The solver keeps full padded node vectors.  Free nodes hold their own entries;
// every node of body b stands for the single unknown psi_b (its direction value is
// p_b, its residual lives in rb[b]); Dirichlet and halo nodes hold zero.  Then
//   (A p)_free = (K p)_free and (A p)_b = sum over the nodes of body b of (K p)_n,
// which is Algorithm 1's assembly of element results into r (interior nodes) and rb
// (body DOFs), and p.Ap = sum_free p (Kp) + sum_b p_b (Ap)_b.
// Every solve runs one kernel per CG iteration (k_step, step.h; the batched solver
// runs it for many systems per launch, batch.h); each block reduces the previous
// launch's per-block partials itself.  Scalars never leave the device; the host polls
// a done flag every few iterations.
#include <dlfcn.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "adjoint.h"
#include "apply.h"
#include "step.h"

namespace mfp {

struct SetupArgs {
  Layout L;
  int nx, ny;
  double x0, y0, hx, hy, inv_hx;
  double U;
  int bc[4];
  double c0x, c0y, c0r;          // circle 0 (cylinder boundary data)
  int phi;                       // velocity potential: body nodes are unknowns of their own
  const double* disp;            // caller displacement (unpadded)
  const int8_t* kind;
  const int8_t* body;
  int8_t* tag;
  double* dx;
  double* dy;
  float* dxf;
  float* dyf;
  double* g;
  double* x;
  double* r;
  double* p0;
  double* p1;
  double* q;
  long long* nfree;
  unsigned long long fixed_mask;  // bit b: body b held at the value fixed[b] (Dirichlet)
  double fixed[MFP_MAX_BODIES];
};

__device__ double side_value(int code, double x, double y, const SetupArgs& a) {
  if (code == MFP_BC_DIRICHLET_UY) return a.U * y;
  if (code == MFP_BC_DIRICHLET_UX) return a.U * x;
  if (code == MFP_BC_DIRICHLET_CYL || code == MFP_BC_DIRICHLET_CYLPHI) {
    const double dx = x - a.c0x, dy = y - a.c0y;
    const double rho2 = dx * dx + dy * dy;
    const double k = a.c0r * a.c0r / rho2;
    return code == MFP_BC_DIRICHLET_CYL ? a.U * dy * (1.0 - k) : a.U * dx * (1.0 + k);
  }
  return 0.0;
}

// Whether node (i, j) belongs to an active cell (a cell whose four nodes do not all
// lie in one body): the domain of the velocity potential.
__device__ bool node_in_domain(const int8_t* __restrict__ body, int nx, int ny, int i, int j) {
  for (int cj = j - 1; cj <= j; ++cj) {
    for (int ci = i - 1; ci <= i; ++ci) {
      if (ci < 0 || cj < 0 || ci >= nx || cj >= ny) continue;
      const long long n0 = (long long)cj * (nx + 1) + ci;
      const int b0 = body[n0];
      if (b0 < 0 || body[n0 + 1] != b0 || body[n0 + nx + 1] != b0 || body[n0 + nx + 2] != b0)
        return true;
    }
  }
  return false;
}

__global__ void k_setup(SetupArgs a) {
  const long long n = a.L.n;
  long long cnt = 0;
  const long long nn = (long long)(a.nx + 1) * (a.ny + 1);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int row = (int)(e / a.L.P), col = (int)(e - (long long)row * a.L.P);
    const int i = column_node(col), j = row - 1;
    int8_t tg = TAG_HALO;
    double dxv = 0.0, dyv = 0.0, gv = 0.0;
    if (i >= 0 && i <= a.nx && j >= 0 && j <= a.ny) {
      const long long nd = (long long)j * (a.nx + 1) + i;
      const int b = a.body ? a.body[nd] : -1;
      const bool left = i == 0 && a.bc[0] != MFP_BC_NATURAL;
      const bool right = i == a.nx && a.bc[1] != MFP_BC_NATURAL;
      const bool bot = j == 0 && a.bc[2] != MFP_BC_NATURAL;
      const bool top = j == a.ny && a.bc[3] != MFP_BC_NATURAL;
      if (b >= 0 && !a.phi && ((a.fixed_mask >> b) & 1ull)) {
        tg = TAG_DIR;  // a body held at a given value: its nodes are Dirichlet nodes
        gv = a.fixed[b];
      } else if (b >= 0) {
        tg = a.phi ? tag_potential_body(b) : (int8_t)(TAG_BODY0 + b);
        if (a.phi && node_in_domain(a.body, a.nx, a.ny, i, j)) ++cnt;
      } else if (left || right || bot || top) {
        tg = TAG_DIR;
        const double x = a.x0 + (double)i * a.hx, y = a.y0 + (double)j * a.hy;
        const int code = bot ? a.bc[2] : top ? a.bc[3] : left ? a.bc[0] : a.bc[1];
        gv = side_value(code, x, y, a);
      } else {
        tg = TAG_FREE;
        ++cnt;
      }
      if (a.disp) {
        dxv = a.disp[nd] * a.inv_hx;
        dyv = a.disp[nd + nn] * a.inv_hx;
      }
    }
    a.tag[e] = tg;
    a.dx[e] = dxv;
    a.dy[e] = dyv;
    if (a.dxf) {
      a.dxf[e] = (float)dxv;
      a.dyf[e] = (float)dyv;
    }
    if (a.g) a.g[e] = gv;
    if (a.x) a.x[e] = 0.0;
    if (a.r) a.r[e] = 0.0;
    if (a.p0) a.p0[e] = 0.0;
    if (a.p1) a.p1[e] = 0.0;
    if (a.q) a.q[e] = 0.0;
  }
  if (a.nfree && cnt) atomicAdd((unsigned long long*)a.nfree, (unsigned long long)cnt);
}

// Per task: constant-stencil flag (footprint of 64 columns x HC+2 rows all free and
// undisplaced) and the set of bodies among the task's owned nodes (none for the
// potential).  One wavefront per task.
__global__ void __launch_bounds__(BLOCK) k_task_meta(Layout L, const int8_t* __restrict__ tag,
                                                     const double* __restrict__ dx,
                                                     const double* __restrict__ dy,
                                                     uint8_t* __restrict__ tplain,
                                                     unsigned long long* __restrict__ tbody) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * WAVES + (threadIdx.x >> 6);
  if (t >= L.ntasks()) return;
  const int m = t % L.nstrip, kc = t / L.nstrip;
  const int HC = L.hc;
  const long long base =
      (long long)(kc * HC) * L.P + (long long)m * 64 + lane + halo_shift(lane, m, L.nstrip);
  int plain = 1;
  unsigned long long bm = 0;
  for (int r = 0; r < HC + 2; ++r) {
    const long long gi = base + (long long)r * L.P;
    const int8_t tg = tag[gi];
    if (tg != TAG_FREE || dx[gi] != 0.0 || dy[gi] != 0.0) plain = 0;
    // (the potential's body tags are negative: no body constraint)
    if (r >= 1 && r <= HC && lane >= 1 && lane <= SW && tg >= TAG_BODY0)
      bm |= 1ull << (tg - TAG_BODY0);
  }
  for (int off = 32; off > 0; off >>= 1) {
    bm |= __shfl_xor(bm, off, 64);
    plain &= __shfl_xor(plain, off, 64);
  }
  if (lane == 0) {
    tplain[t] = (uint8_t)plain;
    tbody[t] = bm;
  }
}

// Caller node vector (node (i, j) at j (nx+1) + i) to and from the padded layout.
template <typename T>
__global__ void k_to_padded(Layout L, const T* __restrict__ src, T* __restrict__ dst) {
  const long long nn = (long long)(L.nx + 1) * (L.ny + 1);
  for (long long nd = blockIdx.x * (long long)blockDim.x + threadIdx.x; nd < nn;
       nd += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(nd / (L.nx + 1)), i = (int)(nd - (long long)j * (L.nx + 1));
    dst[node_index(L, i, j)] = src[nd];
  }
}

template <typename T>
__global__ void k_from_padded(Layout L, const T* __restrict__ src, T* __restrict__ dst) {
  const long long nn = (long long)(L.nx + 1) * (L.ny + 1);
  for (long long nd = blockIdx.x * (long long)blockDim.x + threadIdx.x; nd < nn;
       nd += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(nd / (L.nx + 1)), i = (int)(nd - (long long)j * (L.nx + 1));
    dst[nd] = src[node_index(L, i, j)];
  }
}

// Slots for tiles that own body nodes, numbered in tile order (single block).
__global__ void k_assign_slots(int ntiles, const unsigned long long* __restrict__ tbody,
                               int* __restrict__ tslot, int* __restrict__ nslots) {
  __shared__ int s_scan[BLOCK];
  __shared__ int s_base;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < ntiles; c0 += BLOCK) {
    const int t = c0 + threadIdx.x;
    const int f = (t < ntiles && tbody[t] != 0ull) ? 1 : 0;
    s_scan[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
      const int v = threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0;
      __syncthreads();
      s_scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (t < ntiles) tslot[t] = f ? s_base + s_scan[threadIdx.x] - 1 : -1;
    __syncthreads();
    if (threadIdx.x == BLOCK - 1) s_base += s_scan[BLOCK - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *nslots = s_base;
}

// Apply work list.  The tasks of each strip are cut into segments of consecutive
// chunks (one wavefront marches through one segment) so that every segment costs
// about the same: a constant-stencil task counts 1, a task that evaluates its cells'
// geometry GENERAL_COST (measured ratio of their run times).  The budget is the total
// cost over `target` segments; a segment closes once it reaches the budget or 64
// tasks, so a strip of cost c yields at most floor(c / budget) + 1 + nchunk / 64
// segments and the whole list at most target + nstrip (1 + nchunk / 64) entries (the
// host sizes the table by that bound).
// Placement: wavefront w of a launch of W = 4 G wavefronts reads entries w, w + W, ...;
// its work-group runs on XCD x for w in [x W/8, (x+1) W/8) (see apply_core).  The
// segments, in strip order, are dealt to the 8 XCDs in contiguous runs of equal count,
// each run filling its XCD's entries round by round, so neighbouring strips share an
// L2 and every XCD gets the same share of the work.  Unused entries have length 0.
// Entry: x = strip, y = first chunk | (length << 16), (z, w) = 64-bit mask of the
// segment's constant-stencil tasks.  One block.
constexpr int GENERAL_COST = 4;
constexpr int SEG_MAX_STRIPS = 2048;

__global__ void __launch_bounds__(1024) k_seg_plan(Layout L, const uint8_t* __restrict__ tplain,
                                                   int target, int W, int tabsize,
                                                   int4* __restrict__ segtab) {
  __shared__ int s_off[SEG_MAX_STRIPS];
  __shared__ long long s_red[1024 / 64];
  __shared__ int s_budget, s_total;
  const int nt = L.ntasks(), ns = L.nstrip, nc = L.nchunk;
  for (int i = threadIdx.x; i < tabsize; i += blockDim.x) segtab[i] = make_int4(0, 0, 0, 0);
  long long c = 0;
  for (int t = threadIdx.x; t < nt; t += blockDim.x) c += tplain[t] ? 1 : GENERAL_COST;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += s_red[i];
    long long b = (tot + target - 1) / target;
    if (b < GENERAL_COST) b = GENERAL_COST;
    s_budget = (int)(b < (1 << 30) ? b : (1 << 30));
  }
  __syncthreads();
  const int budget = s_budget;
  // with `first` >= 0, segment j (strip order, from `first`) goes to pos(j)
  const int per = W / 8;  // entries per XCD and round
  auto walk = [&](int m, int first, int total) -> int {
    int cnt = 0, acc = 0, len = 0, kc0 = 0;
    unsigned long long mask = 0ull;
    for (int kc = 0; kc < nc; ++kc) {
      const int pl = tplain[kc * ns + m];
      acc += pl ? 1 : GENERAL_COST;
      if (pl) mask |= 1ull << len;
      ++len;
      if (acc >= budget || len == 64 || kc == nc - 1) {
        if (first >= 0) {
          const int j = first + cnt;
          const int q = total / 8, rem = total % 8;
          // XCD x holds segments [x q + min(x, rem), ...)
          const int x = j < rem * (q + 1) ? j / (q + 1) : rem + (j - rem * (q + 1)) / (q > 0 ? q : 1);
          const int i = j - (x * q + (x < rem ? x : rem));
          const long long pos = (long long)(i / per) * W + (long long)x * per + i % per;
          if (pos < tabsize)
            segtab[pos] = make_int4(m, kc0 | (len << 16), (int)(mask & 0xffffffffull),
                                    (int)(mask >> 32));
        }
        ++cnt;
        acc = 0;
        len = 0;
        mask = 0ull;
        kc0 = kc + 1;
      }
    }
    return cnt;
  };
  for (int m = threadIdx.x; m < ns; m += blockDim.x) s_off[m] = walk(m, -1, 0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int m = 0; m < ns; ++m) {
      const int v = s_off[m];
      s_off[m] = acc;
      acc += v;
    }
    s_total = acc;
  }
  __syncthreads();
  const int total = s_total;
  for (int m = threadIdx.x; m < ns; m += blockDim.x) walk(m, s_off[m], total);
}

// w = g + T x as a full nodal vector (free: x, Dirichlet: g, body b: psi_b of the
// current iterate; the potential's body nodes, negative tags: x).
template <typename T>
__global__ void k_form_w(long long n, const int8_t* __restrict__ tag,
                         const double* __restrict__ x, const double* __restrict__ g,
                         const DevState* __restrict__ st, T* __restrict__ w) {
  const double* xb = st->xb[st->iters & 1];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int8_t tg = tag[e];
    double v = 0.0;
    if (tag_own(tg))
      v = x[e];
    else if (tg == TAG_DIR)
      v = g[e];
    else if (tg >= TAG_BODY0)
      v = xb[tg - TAG_BODY0];
    w[e] = (T)v;
  }
}

// r = -q at free nodes (q is zero elsewhere) when write_r; per-block partials of q.q.
__global__ void __launch_bounds__(BLOCK) k_resid(long long n, const double* __restrict__ q,
                                                 double* __restrict__ r, double* __restrict__ part,
                                                 int write_r) {
  __shared__ double s_red[BLOCK / 64];
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double v = q[e];
    if (write_r) r[e] = -v;
    acc += v * v;
  }
  const double bs = block_sum(acc, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// Single block.  Body sums of the last plain apply (q = K w, w = g + T x), then with
// rr = ||b - A x||^2 = q.q over free nodes + sum_b qb^2:
// mode 0: CG state for a start from the current iterate (x, xb of the current slot):
//         rb = -qb, p_b = 0 and r.r = 1 in the "previous" slot so that the first
//         direction is the residual; the first call also records rr0; the stopping
//         threshold is stop_abs if positive, else rtol2 * rr0;
// mode 1: record rr only (true residual at the end);
// mode 2: record rr and rb = -qb (outer residual of iterative refinement).
__global__ void __launch_bounds__(BLOCK) k_resid_finalize(const double* __restrict__ part,
                                                          int G2, const double* __restrict__ bpart,
                                                          const int* __restrict__ nslots,
                                                          DevState* st, int nb, int mode,
                                                          double rtol2, double stop_abs) {
  __shared__ double s_red[BLOCK / 64];
  __shared__ double s_qb[MFP_MAX_BODIES];
  body_sums(bpart, nslots, nb, s_qb);
  double s = 0.0;
  for (int i = threadIdx.x; i < G2; i += BLOCK) s += part[i];
  s = block_sum(s, s_red);
  if (threadIdx.x == 0) {
    // body residuals: right-hand side of the body rows minus their sums of K w
    double rbr = 0.0;
    for (int b = 0; b < nb; ++b) {
      st->qb[b] = s_qb[b];
      const double v = st->bb[b] - s_qb[b];
      rbr += v * v;
    }
    const double rr = s + rbr;
    st->rr_true = rr;
    if (mode == 0) {
      const int it = (int)(st->iters & 1);
      for (int b = 0; b < nb; ++b) {
        st->xb[0][b] = st->xb[it][b];
        st->rb[0][b] = st->bb[b] - s_qb[b];
        st->pb[1][b] = 0.0;
      }
      st->rb_rr[0] = rbr;
      st->rr[1] = 1.0;
      if (st->rr0 == 0.0) st->rr0 = rr;
      st->rr_stop = stop_abs > 0.0 ? stop_abs : rtol2 * st->rr0;
      st->iters = 0;
      st->done = 0;
    } else if (mode == 2) {
      for (int b = 0; b < nb; ++b) st->rb[0][b] = st->bb[b] - s_qb[b];
    }
  }
}

// Reliable update of the mixed-precision solve: x64 += e32 (all nodes; only free
// entries are ever read), e32 = 0, and the body corrections move from the inner
// state (slot k&1) to the outer one.
__global__ void k_ir_update(long long n, double* __restrict__ x64, float* __restrict__ e32,
                            DevState* outer, DevState* in, int nb, int slot) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    x64[e] += (double)e32[e];
    e32[e] = 0.f;
  }
  if (blockIdx.x == 0 && (int)threadIdx.x < nb) {
    const int b = threadIdx.x;
    outer->xb[outer->iters & 1][b] += in->xb[slot][b];
    in->xb[slot][b] = 0.0;
  }
}

// psi (unpadded) from the padded unknowns; Q and CoPFI from the pair.
__global__ void k_output(Layout L, int nx, int ny, const int8_t* __restrict__ tag,
                         const double* __restrict__ x, const double* __restrict__ g,
                         DevState* st, double* __restrict__ psi, int lo, int hi, double U,
                         double ylo, double yhi) {
  const long long nn = (long long)(nx + 1) * (ny + 1);
  const double* xb = st->xb[st->iters & 1];
  for (long long nd = blockIdx.x * (long long)blockDim.x + threadIdx.x; nd < nn;
       nd += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(nd / (nx + 1)), i = (int)(nd - (long long)j * (nx + 1));
    const long long e = node_index(L, i, j);
    const int8_t tg = tag[e];
    psi[nd] = tg == TAG_FREE ? x[e] : tg == TAG_DIR ? g[e] : xb[tg - TAG_BODY0];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && lo >= 0 && hi >= 0) {
    st->Q = xb[hi] - xb[lo];
    st->copfi = st->Q / (U * (yhi - ylo));
  }
}

// The potential (unpadded): unknowns from x, Dirichlet nodes from g, NaN at nodes of no
// active cell (inside a body).
__global__ void k_output_phi(Layout L, int nx, int ny, const int8_t* __restrict__ tag,
                             const int8_t* __restrict__ body, const double* __restrict__ x,
                             const double* __restrict__ g, double* __restrict__ phi) {
  const long long nn = (long long)(nx + 1) * (ny + 1);
  for (long long nd = blockIdx.x * (long long)blockDim.x + threadIdx.x; nd < nn;
       nd += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(nd / (nx + 1)), i = (int)(nd - (long long)j * (nx + 1));
    const long long e = node_index(L, i, j);
    const int8_t tg = tag[e];
    double v;
    if (tg == TAG_DIR)
      v = g[e];
    else if (tg < TAG_FREE && !node_in_domain(body, nx, ny, i, j))
      v = __builtin_nan("");
    else
      v = x[e];
    phi[nd] = v;
  }
}

// Surface tangential velocity samples (section "Velocity Field and Surface
// Tangential Velocity"): u_t = (psi_c - psi_b) / d_nc on each edge joining two nodes
// snapped to the same body, in every active cell with a fluid node.  psi_c is the mean
// nodal psi of the cell, d_nc the distance from the mean of its displaced nodes to the
// line through the edge, theta the polar angle of the edge midpoint.  The items are the
// cells of every body's box, body after body and in cell-id order within a box; three
// passes (samples per block, one block scanning the block counts, a write pass that
// recounts and scans within its block) keep the output order (body, cell, local edge)
// without atomics.
struct SampleArgs {
  int nx, ny, nb;
  double x0, y0, hx, hy, hmax;
  const mfp_circle* circ;
  const int* boxes;  // per body: ci0, ci1, cj0, cj1 (cells)
  const double* disp;
  const int8_t* kind;
  const int8_t* body;
  const double* psi;
  const DevState* st;
  double* samples;
  int8_t* sbody;
  int cap;
  int* count;
  long long items;                        // cells of all boxes, body after body
  long long first[MFP_MAX_BODIES + 1];    // first item of each body's box
  int* boff;                              // per block: sample count, then offset
};

constexpr int SMP_ITEMS = 4;                     // consecutive items per thread
constexpr int SMP_CHUNK = BLOCK * SMP_ITEMS;     // items per block
constexpr int SMP_MAX_BLOCKS = 1 << 16;          // up to 2^26 box cells

// Samples of item it (body b, cell c of its box in cell-id order), in edge order;
// (theta, u_t) into th/ut when they are non-null.  Returns the count (0..4).
__device__ int item_samples(const SampleArgs& a, long long it, int* bout, double* th,
                            double* ut) {
  int b = 0;
  while (b + 1 < a.nb && it >= a.first[b + 1]) ++b;
  *bout = b;
  const long long c = it - a.first[b];
  const int ci0 = a.boxes[4 * b], ci1 = a.boxes[4 * b + 1];
  const int cj0 = a.boxes[4 * b + 2];
  const int bw = ci1 - ci0 + 1;
  const int ci = ci0 + (int)(c % bw), cj = cj0 + (int)(c / bw);
  const long long nn = (long long)(a.nx + 1) * (a.ny + 1);
  const long long n0 = (long long)cj * (a.nx + 1) + ci;
  const long long nd[4] = {n0, n0 + 1, n0 + a.nx + 2, n0 + a.nx + 1};
  const int bb0 = a.body[nd[0]];
  const bool inside =
      bb0 >= 0 && a.body[nd[1]] == bb0 && a.body[nd[2]] == bb0 && a.body[nd[3]] == bb0;
  bool fluid = false;
  for (int k = 0; k < 4; ++k) fluid |= a.kind[nd[k]] == MFP_FLUID;
  if (inside || !fluid) return 0;
  double X[4], Y[4], ps[4];
  const int oi[4] = {0, 1, 1, 0}, oj[4] = {0, 0, 1, 1};
  for (int k = 0; k < 4; ++k) {
    X[k] = a.x0 + (double)(ci + oi[k]) * a.hx + a.disp[nd[k]];
    Y[k] = a.y0 + (double)(cj + oj[k]) * a.hy + a.disp[nd[k] + nn];
    ps[k] = a.psi[nd[k]];
  }
  const double gx = 0.25 * ((X[0] + X[1]) + (X[2] + X[3]));
  const double gy = 0.25 * ((Y[0] + Y[1]) + (Y[2] + Y[3]));
  const double psic = 0.25 * ((ps[0] + ps[1]) + (ps[2] + ps[3]));
  const double psib = a.st->xb[a.st->iters & 1][b];
  int cnt = 0;
  for (int k = 0; k < 4; ++k) {
    const int k2 = (k + 1) & 3;
    if (a.kind[nd[k]] == MFP_SNAPPED && a.kind[nd[k2]] == MFP_SNAPPED && a.body[nd[k]] == b &&
        a.body[nd[k2]] == b) {
      const double ex = X[k2] - X[k], ey = Y[k2] - Y[k];
      const double len = sqrt(ex * ex + ey * ey);
      if (len > 1e-12 * a.hmax) {
        if (th) {
          const double dnc = fabs(ex * (gy - Y[k]) - ey * (gx - X[k])) / len;
          const double mx = 0.5 * (X[k] + X[k2]), my = 0.5 * (Y[k] + Y[k2]);
          th[cnt] = atan2(my - a.circ[b].cy, mx - a.circ[b].cx);
          ut[cnt] = (psic - psib) / dnc;
        }
        ++cnt;
      }
    }
  }
  return cnt;
}

// Exclusive scan of one int per thread over the block; *sum gets the block total.
__device__ int block_exscan_int(int v, int* s_scan, int* sum) {
  const int tid = threadIdx.x;
  s_scan[tid] = v;
  __syncthreads();
  for (int off = 1; off < BLOCK; off <<= 1) {
    const int u = tid >= off ? s_scan[tid - off] : 0;
    __syncthreads();
    s_scan[tid] += u;
    __syncthreads();
  }
  const int incl = s_scan[tid];
  *sum = s_scan[BLOCK - 1];
  __syncthreads();
  return incl - v;
}

// Pass 1: samples per block of SMP_CHUNK items.
__global__ void __launch_bounds__(BLOCK) k_samples_count(SampleArgs a) {
  __shared__ int s_scan[BLOCK];
  const long long i0 = (long long)blockIdx.x * SMP_CHUNK + (long long)threadIdx.x * SMP_ITEMS;
  int cnt = 0, b;
  for (int q = 0; q < SMP_ITEMS; ++q)
    if (i0 + q < a.items) cnt += item_samples(a, i0 + q, &b, nullptr, nullptr);
  int sum;
  (void)block_exscan_int(cnt, s_scan, &sum);
  if (threadIdx.x == 0) a.boff[blockIdx.x] = sum;
}

// Pass 2 (one block): block counts -> offsets; the total into *count.
__global__ void __launch_bounds__(BLOCK) k_samples_scan(SampleArgs a, int nblk) {
  __shared__ int s_scan[BLOCK];
  const int per = (nblk + BLOCK - 1) / BLOCK;
  const int b0 = threadIdx.x * per;
  int loc = 0;
  for (int k = 0; k < per; ++k)
    if (b0 + k < nblk) loc += a.boff[b0 + k];
  int sum;
  int off = block_exscan_int(loc, s_scan, &sum);
  for (int k = 0; k < per; ++k)
    if (b0 + k < nblk) {
      const int c = a.boff[b0 + k];
      a.boff[b0 + k] = off;
      off += c;
    }
  if (threadIdx.x == 0) *a.count = sum;
}

// Pass 3: every block writes its samples from its offset, in item and edge order.
__global__ void __launch_bounds__(BLOCK) k_samples_write(SampleArgs a) {
  __shared__ int s_scan[BLOCK];
  const long long i0 = (long long)blockIdx.x * SMP_CHUNK + (long long)threadIdx.x * SMP_ITEMS;
  int cnt = 0, b;
  for (int q = 0; q < SMP_ITEMS; ++q)
    if (i0 + q < a.items) cnt += item_samples(a, i0 + q, &b, nullptr, nullptr);
  int sum;
  int o = a.boff[blockIdx.x] + block_exscan_int(cnt, s_scan, &sum);
  for (int q = 0; q < SMP_ITEMS; ++q) {
    if (i0 + q >= a.items) break;
    double th[4], ut[4];
    const int k = item_samples(a, i0 + q, &b, th, ut);
    for (int s = 0; s < k; ++s, ++o)
      if (o < a.cap) {
        a.samples[2 * o] = th[s];
        a.samples[2 * o + 1] = ut[s];
        a.sbody[o] = (int8_t)b;
      }
  }
}

// ---------------------------------------------------------------------------------
// Workspace and host driver
// ---------------------------------------------------------------------------------
constexpr int GMAX = 2048;  // max blocks of the reduction kernels
// Launches whose CG scalars are kept for the condition estimate (256 KiB).
constexpr long long HIST_CAP = 16384;

// Wavefronts of the one-kernel CG iteration k_step<T, hc> resident on the current
// device at once (0 when the runtime cannot say).
template <typename T>
static int step_resident_waves(int hc = 4, int kst = 0) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const void* f =
      kst ? (hc == 8   ? reinterpret_cast<const void*>(&k_step<T, 8, false, true, true>)
             : hc == 5 ? reinterpret_cast<const void*>(&k_step<T, 5, false, true, true>)
                       : reinterpret_cast<const void*>(&k_step<T, 4, false, true, true>))
          : (hc == 8   ? reinterpret_cast<const void*>(&k_step<T, 8, false, true, false>)
             : hc == 5 ? reinterpret_cast<const void*>(&k_step<T, 5, false, true, false>)
                       : reinterpret_cast<const void*>(&k_step<T, 4, false, true, false>));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, BLOCK, 0) != hipSuccess) return 0;
  return per_cu * cus * WAVES;
}

// Blocks of the one-kernel iteration: as many as stay resident at once (so that no
// second round of work-groups trails the first), at most one task per wavefront and at
// most 1024 (the next launch reduces one partial per block); a multiple of 8.
template <typename T>
static int step_blocks(const Layout& L, int kst = 0, int forced = 0) {
  const long long need = (((long long)L.ntasks() + WAVES - 1) / WAVES + 7) & ~7LL;
  long long g = forced > 0 ? forced : step_resident_waves<T>(L.hc, kst) / WAVES;
  g &= ~7LL;
  if (g < 8) g = 8;
  if (g > need) g = need;
  if (g > 1024) g = 1024;
  return (int)g;
}

// ---- one task per wavefront, geometry tasks on distinct SIMDs --------------------
// When the tasks fit the wavefronts that a launch of 8-wavefront blocks keeps resident
// with one block per CU, every wavefront runs one task and the launch lasts as long as
// its busiest SIMD.  A task that evaluates geometry issues several times the vector
// instructions of a constant-stencil task, and two on one SIMD take turns at its
// issue port.  The table below deals the tasks so that no SIMD holds two geometry tasks
// while another holds none, and gives every XCD an eighth of each kind.  It relies on
// where the hardware places work-groups and wavefronts (checked on the target with
// the hardware-id register): work-group k runs on XCD k mod 8, a 512-thread group
// that fills a CU is alone there, and its wavefronts w and w + 4 share SIMD w mod 4.
// Were the placement different, the result would be the same, only slower.
constexpr int PAIR_SLOTS = 8 * 1024;  // table entries: 8 wavefronts x up to 1024 CUs

// Blocks of the table launch for k_step<T, hc> (with stored entries: kst) - the
// device's CU count, one block per CU (where two would fit, the dispatcher still deals
// the first block of every CU before any second one) - or 0 when the table does not
// apply: the 8-wavefront kernel does not fit a CU, needs scratch memory (spilled
// registers), or there are more tasks than its wavefronts.
template <typename T, bool KST>
static const void* table_kernel(int hc, bool odd) {
  if (odd)
    return hc == 8   ? reinterpret_cast<const void*>(&k_step<T, 8, false, true, KST, 8>)
           : hc == 5 ? reinterpret_cast<const void*>(&k_step<T, 5, false, true, KST, 8>)
                     : reinterpret_cast<const void*>(&k_step<T, 4, false, true, KST, 8>);
  return hc == 8   ? reinterpret_cast<const void*>(&k_step<T, 8, false, false, KST, 8>)
         : hc == 5 ? reinterpret_cast<const void*>(&k_step<T, 5, false, false, KST, 8>)
                   : reinterpret_cast<const void*>(&k_step<T, 4, false, false, KST, 8>);
}

template <typename T>
static int pair_blocks(int hc, int ntask, bool kst) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (cus <= 0 || cus % 8 != 0 || 8 * cus > PAIR_SLOTS || ntask > 8 * cus) return 0;
  for (int odd = 0; odd < 2; ++odd) {
    const void* f = kst ? table_kernel<T, true>(hc, odd) : table_kernel<T, false>(hc, odd);
    hipFuncAttributes fa;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 8 * 64, 0) != hipSuccess ||
        per_cu < 1 || hipFuncGetAttributes(&fa, f) != hipSuccess || fa.localSizeBytes != 0)
      return 0;
  }
  return cus;
}

// The table for `cus` blocks of 8 wavefronts: tab[8 k + w] is the task of wavefront w
// of block k, or -1, and its flags (bit 0: constant stencil, plain[t] != 0; bit 1: the
// task holds body nodes, tbody[t] != 0; bits 2..15: its body-sum slot tslot[t] + 1;
// bits 16..30: its stored-entry slab tgeo[t] + 1, tgeo may be NULL), so that the
// kernel loads no flags before the task's data.  XCD x takes the
// x-th eighth of the geometry tasks and of the others (each a run of neighbouring
// tasks in task order); its geometry tasks go one per SIMD (a second one per SIMD only
// when they outnumber its SIMDs), its other tasks first to the SIMDs left empty, then
// as second tasks of the SIMDs without a geometry task, then of the rest.  False if
// some XCD's share exceeds its wavefronts.
static bool pair_table(const uint8_t* plain, const unsigned long long* tbody, const int* tslot,
                       const int* tgeo, int ntask, int cus, int2* tab) {
  if (ntask >= (1 << 14) - 1) return false;  // slot and slab fields
  std::vector<int> geo, pl;
  for (int t = 0; t < ntask; ++t) (plain[t] ? pl : geo).push_back(t);
  const int S = 4 * (cus / 8);  // SIMDs per XCD
  const long long ng = (long long)geo.size(), np = (long long)pl.size();
  for (int e = 0; e < 8 * cus; ++e) tab[e] = make_int2(-1, 1);
  std::vector<int> first(S), second(S);
  for (int x = 0; x < 8; ++x) {
    const int g0 = (int)(ng * x / 8), g1 = (int)(ng * (x + 1) / 8);
    const int p0 = (int)(np * x / 8), p1 = (int)(np * (x + 1) / 8);
    if ((g1 - g0) + (p1 - p0) > 2 * S) return false;
    std::fill(first.begin(), first.end(), -1);
    std::fill(second.begin(), second.end(), -1);
    for (int i = g0; i < g1; ++i) {
      const int u = i - g0;
      (u < S ? first[u] : second[u - S]) = geo[i];
    }
    int k = p0;
    for (int u = 0; u < S && k < p1; ++u)
      if (first[u] < 0) first[u] = pl[k++];
    for (int u = S - 1; u >= 0 && k < p1; --u)
      if (second[u] < 0) second[u] = pl[k++];
    if (k != p1) return false;
    for (int u = 0; u < S; ++u) {
      const int blk = x + 8 * (u / 4), w = u % 4;
      tab[8 * blk + w].x = first[u];
      tab[8 * blk + w + 4].x = second[u];
    }
  }
  // every task exactly once; the flags
  std::vector<uint8_t> seen(ntask, 0);
  for (int e = 0; e < 8 * cus; ++e) {
    const int t = tab[e].x;
    if (t >= 0 && t < ntask)
      tab[e].y = (plain[t] ? 1 : 0) | (tbody[t] ? 2 : 0) | ((tslot[t] + 1) << 2) |
                 ((tgeo ? tgeo[t] + 1 : 0) << 16);
    if (t < -1 || t >= ntask || (t >= 0 && seen[t]++)) return false;
  }
  for (int t = 0; t < ntask; ++t)
    if (!seen[t]) return false;
  return true;
}

// Segments for a single solve: about as many as the solve loop's kernel keeps
// resident, less the per-strip slack of the segment bound, so that the whole list runs
// in one round of wavefronts.
static int single_target(const Layout& L, int precision) {
  const int wres = precision == MFP_FP64 ? step_resident_waves<double>(L.hc)
                                         : step_resident_waves<float>(L.hc);
  if (wres <= 0) return L.ntasks();
  int t = wres - L.nstrip * (L.nchunk / 64 + 1);
  if (t < wres / 2) t = wres / 2;
  return t > 0 ? t : 1;
}

// Size of the apply work list for a segment target (see k_seg_plan) and the launch
// that covers it: at most 1024 blocks, a multiple of 8 (XCD-aware order); with more
// entries than wavefronts, each wavefront takes every W-th entry.
struct SegPlan {
  int target = 1, tabsize = 32, G = 8;
};

static SegPlan seg_plan(const Layout& L, int target) {
  SegPlan p;
  const long long nt = L.ntasks();
  if (target < 1) target = 1;
  long long cap = (long long)target + (long long)L.nstrip * (L.nchunk / 64 + 1);
  if (cap > nt) cap = nt;
  long long G = (cap + WAVES - 1) / WAVES;
  G = (G + 7) & ~7LL;
  if (G > 1024) G = 1024;
  const long long W = WAVES * G;
  // rounds so that every XCD's share, ceil(cap / 8), fits in its W/8 entries per round
  const long long rounds = ((cap + 7) / 8 + W / 8 - 1) / (W / 8);
  p.target = target;
  p.tabsize = (int)(rounds * W);
  p.G = (int)G;
  return p;
}

// Schedule of the one-kernel iteration of a single solve.
struct Schedule {
  int hc = 4;       // node rows per task: 4, 5 or 8
  int kst = 0;      // 1: the geometry tasks read stored element entries (k_elem_coef)
  int stream = -1;  // -1: by working-set size; 0: cached stores; 1: streaming stores
  int blocks = 0;   // blocks per launch; 0: as many as stay resident
  int cells = 0;    // 1: the stored entries come from a caller's per-cell table (FP64
                    //    slabs kept for the residuals in every precision)
};

// Values per task slab of stored element entries (cell rows x entries x lanes).
inline size_t kslab_rows(int hc) { return (size_t)(hc + 1) * KCOEF * 64; }

struct SolveWs {
  Layout L;
  SegPlan sp;     // apply work list and launch size
  int8_t* tag;
  double *dx, *dy, *g, *x, *r, *p0, *p1, *q;
  double *r1, *q1;   // second residual / K p slots of the one-kernel iteration
  float *dxf, *dyf, *xf, *rf, *p0f, *p1f, *qf;
  float *r1f, *q1f;
  uint8_t* tplain;
  unsigned long long* tbody;
  int* tslot;
  int* nslots;
  mutable int nslots_h = 0;  // host copy of *nslots (read once after setup)
  int4* segtab;   // apply work list (k_seg_plan)
  double* part;
  double* part2;
  double* part3;  // batched refinement: partials of the FP64 residual
  double* bpart;
  size_t bstride;   // per-slot body sums: parity slot 1 starts at bpart + bstride
  double* spart;    // one-kernel iteration partials, 2 slots x 4 x GMAX
  double* hist;     // CG scalars per launch (alpha_{j-1}, beta_j), HIST_CAP launches
  DevState* st;
  DevState* st2;  // inner (FP32) solver state
  long long* nfree;
  mfp_circle* circ;
  int* boxes;
  int* count;
  int* sboff;     // surface samples: per-block counts / offsets
  int sboff_n = 0;
  int phi = 0;    // velocity-potential solve: body nodes are unknowns, no body constraint
  Schedule sc;    // the iteration's schedule (task rows, element mode, stores, blocks)
  int* tgeo = nullptr;      // stored element entries: per task its slab or -1
  int* ngeo = nullptr;      // number of slabs in use
  double* kc64 = nullptr;   // slabs for an FP64 iteration
  float* kc32 = nullptr;    // slabs for an FP32 iteration
  const double* cellcoef = nullptr;  // per-cell element entries given by the caller
  unsigned long long fixed_mask = 0;  // bodies held at given values (Dirichlet), bit b
  double fixed[MFP_MAX_BODIES] = {};
  int2* wtask = nullptr;         // one task per wavefront (pair_table), PAIR_SLOTS entries
  mutable int pair_blocks = 0;   // blocks of the launch that uses it; 0: table not built
};

// Task height of a single solve's layout.  The FP32 iteration with 8-row tasks uses
// about the registers of the FP64 one with 4-row tasks (two wavefronts per SIMD instead
// of four) and has half the tasks: measured 56.8 vs 60.8 us per launch at 4096x2048,
// but 17.0 vs 15.3 us at 1024x512, where 4-row tasks already give fewer tasks than
// resident wavefronts.  So 8 rows for FP32 once the 4-row layout has at least 8192
// tasks (twice the 4096 wavefronts of 4-row FP32 tasks that 256 CUs hold), else 4.
static int solve_hc(const mfp_grid* g, int precision) {
  if (precision != MFP_FP32 && precision != MFP_FP32_IR) {
    // FP64: 5-row tasks when they fit the resident wavefronts in one round and 4-row
    // tasks do not (a wavefront with a second task doubles the launch's tail)
    const int w = step_resident_waves<double>(4);
    if (w > 0 && make_layout(g->nx, g->ny).ntasks() > w &&
        make_layout(g->nx, g->ny, 5).ntasks() <= step_resident_waves<double>(5))
      return 5;
    return 4;
  }
  return make_layout(g->nx, g->ny).ntasks() >= 8192 ? 8 : 4;
}

// ---- tuning cache ----------------------------------------------------------------
// A text file: the one named by MFP_TUNE_CACHE, else tune_cache.txt beside this
// library (MFP_TUNE_CACHE=none: no cache, built-in rules only).  One entry per line
// (written by the package's tuner, '#' starts a comment):
//   arch nx ny precision batched task_rows element_mode store_mode launch_blocks
//        tasks_per_wave iters_per_launch
// with the fields of mfp_solver_opts (0 = automatic) and, for batched entries, the
// batched solver's tasks per wavefront and launches per replayed block.  Read again
// whenever the file's modification time changes.
struct TuneEntry {
  std::string arch;
  int nx = 0, ny = 0, precision = 0, batched = 0;
  int task_rows = 0, element_mode = 0, store_mode = 0, launch_blocks = 0;
  int tasks_per_wave = 0, iters_per_launch = 0;
};

static std::mutex g_tune_mu;

static std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

static std::string tune_cache_path() {
  const char* env = std::getenv("MFP_TUNE_CACHE");
  if (env) return (!*env || std::strcmp(env, "none") == 0) ? std::string() : std::string(env);
  Dl_info info;
  if (!dladdr(reinterpret_cast<const void*>(&tune_cache_path), &info) || !info.dli_fname)
    return "";
  std::string lib = info.dli_fname;
  const size_t sl = lib.rfind('/');
  return (sl == std::string::npos ? std::string(".") : lib.substr(0, sl)) + "/tune_cache.txt";
}

// The cache entry for this device, grid, precision and solver kind (false if none).
static bool tuned_entry(const mfp_grid* g, int precision, int batched, TuneEntry* out) {
  const std::string path_s = tune_cache_path();
  if (path_s.empty()) return false;
  const char* path = path_s.c_str();
  static std::vector<TuneEntry> entries;
  static std::string loaded_path, arch;
  static long long loaded_mtime = -1;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  struct stat sb;
  if (stat(path, &sb) != 0) return false;
  const long long mt = (long long)sb.st_mtime * 1000000000LL + (long long)sb.st_mtim.tv_nsec;
  if (loaded_path != path || mt != loaded_mtime) {
    entries.clear();
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
      const size_t h = line.find('#');
      if (h != std::string::npos) line.resize(h);
      std::istringstream is(line);
      TuneEntry e;
      if (is >> e.arch >> e.nx >> e.ny >> e.precision >> e.batched >> e.task_rows >>
          e.element_mode >> e.store_mode >> e.launch_blocks >> e.tasks_per_wave >>
          e.iters_per_launch)
        entries.push_back(e);
    }
    loaded_path = path;
    loaded_mtime = mt;
  }
  if (arch.empty()) arch = device_arch();
  for (auto it = entries.rbegin(); it != entries.rend(); ++it)  // the last entry wins
    if (it->arch == arch && it->nx == g->nx && it->ny == g->ny &&
        it->precision == precision && it->batched == batched) {
      *out = *it;
      return true;
    }
  return false;
}

// Schedule fields (0 = automatic) applied over sc; false for a value out of range.
static bool apply_schedule_fields(int task_rows, int element_mode, int store_mode,
                                  int launch_blocks, Schedule* sc) {
  if (task_rows != 0 && task_rows != 4 && task_rows != 5 && task_rows != 8) return false;
  if (element_mode < 0 || element_mode > 2 || store_mode < 0 || store_mode > 2) return false;
  if (launch_blocks < 0 || launch_blocks > 1024 || (launch_blocks & 7) != 0) return false;
  if (task_rows) sc->hc = task_rows;
  if (element_mode) sc->kst = element_mode == 2 ? 1 : 0;
  if (store_mode) sc->stream = store_mode == 2 ? 1 : 0;
  if (launch_blocks) sc->blocks = launch_blocks;
  return true;
}

// Built-in rules, then the tuning cache, then the caller's explicit fields.
static int resolve_schedule(const mfp_grid* g, int precision, const mfp_solver_opts* o,
                            Schedule* out) {
  Schedule sc;
  sc.hc = solve_hc(g, precision);
  TuneEntry e;
  if (tuned_entry(g, precision, 0, &e))
    (void)apply_schedule_fields(e.task_rows, e.element_mode, e.store_mode, e.launch_blocks, &sc);
  if (o && !apply_schedule_fields(o->task_rows, o->element_mode, o->store_mode,
                                  o->launch_blocks, &sc)) {
    set_error("invalid schedule: task_rows 0/4/5/8, element_mode and store_mode 0..2, "
              "launch_blocks a multiple of 8 up to 1024");
    return MFP_E_ARG;
  }
  *out = sc;
  return MFP_OK;
}

static size_t solve_layout(const mfp_grid* g, int nb, int precision, void* base, SolveWs* out,
                           const Schedule* sched = nullptr) {
  Bump bp(base);
  SolveWs w{};
  if (sched) w.sc = *sched;
  w.L = make_layout(g->nx, g->ny, w.sc.hc);
  const size_t n = (size_t)w.L.n;
  const int nt = w.L.ntasks();
  w.tag = bp.take<int8_t>(n);
  w.dx = bp.take<double>(n);
  w.dy = bp.take<double>(n);
  w.g = bp.take<double>(n);
  w.x = bp.take<double>(n);
  w.r = bp.take<double>(n);
  w.p0 = bp.take<double>(n);
  w.p1 = bp.take<double>(n);
  w.q = bp.take<double>(n);
  w.r1 = bp.take<double>(n);
  w.q1 = bp.take<double>(n);
  if (precision != MFP_FP64) {
    w.dxf = bp.take<float>(n);
    w.dyf = bp.take<float>(n);
    w.xf = bp.take<float>(n);
    w.rf = bp.take<float>(n);
    w.p0f = bp.take<float>(n);
    w.p1f = bp.take<float>(n);
    w.qf = bp.take<float>(n);
    w.r1f = bp.take<float>(n);
    w.q1f = bp.take<float>(n);
  }
  w.tplain = bp.take<uint8_t>(nt);
  w.tbody = bp.take<unsigned long long>(nt);
  w.tslot = bp.take<int>(nt);
  w.nslots = bp.take<int>(1);
  w.segtab = bp.take<int4>((size_t)nt + 4096);
  w.part = bp.take<double>(GMAX);
  w.part2 = bp.take<double>(GMAX);
  w.part3 = bp.take<double>(GMAX);
  // at least 64 slots: the body reductions read the first 64 before the slot count
  w.bstride = (size_t)(nt > 64 ? nt : 64) * (nb > 0 ? nb : 1);
  w.bpart = bp.take<double>(2 * w.bstride);
  w.spart = bp.take<double>(2 * 4 * GMAX);
  w.hist = bp.take<double>(2 * (size_t)HIST_CAP);
  w.st = bp.take<DevState>(1);
  w.st2 = bp.take<DevState>(1);
  w.nfree = bp.take<long long>(1);
  w.circ = bp.take<mfp_circle>(nb > 0 ? nb : 1);
  w.boxes = bp.take<int>(4 * (nb > 0 ? nb : 1));
  w.count = bp.take<int>(1);
  w.wtask = bp.take<int2>(PAIR_SLOTS);
  if (w.sc.kst) {
    // every task could be a geometry task
    w.tgeo = bp.take<int>(nt);
    w.ngeo = bp.take<int>(1);
    const size_t slabs = (size_t)nt * kslab_rows(w.L.hc);
    if (precision == MFP_FP64 || w.sc.cells) w.kc64 = bp.take<double>(slabs);
    if (precision != MFP_FP64) w.kc32 = bp.take<float>(slabs);
  }
  {
    // surface samples: at most nb boxes of at most nx ny cells each
    const long long items = (long long)(nb > 0 ? nb : 0) * g->nx * g->ny;
    const long long blk = (items + SMP_CHUNK - 1) / SMP_CHUNK + 1;
    w.sboff_n = (int)(blk < SMP_MAX_BLOCKS ? blk : SMP_MAX_BLOCKS);
    w.sboff = bp.take<int>((size_t)w.sboff_n);
  }
  if (out) {
    if (base) w.sp = seg_plan(w.L, single_target(w.L, precision));
    *out = w;
  }
  return bp.off + 256;
}

// Streaming kernels: about 8 elements per thread, at most 1024 blocks, so that the
// next kernel's per-block reduction of these partials stays small.
static int grid_blocks(long long n) {
  long long b = (n + 8 * BLOCK - 1) / (8 * BLOCK);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

// Streaming kernels of the single-system CG loop (update, residual, refinement):
// about two elements per thread, so that each thread's operands are requested before
// the block forms its scalars, and at most 1024 blocks, so that the next kernel's
// reduction of the per-block partials stays small.
static int loop_blocks(long long n) {
  long long b = (n + 2 * BLOCK - 1) / (2 * BLOCK);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
static ApplyArgs<T> make_apply_args(const SolveWs& w, const mfp_grid& g, int nb, const T* dx,
                                    const T* dy) {
  ApplyArgs<T> a{};
  a.P = w.L.P;
  a.nstrip = w.L.nstrip;
  a.segtab = w.segtab;
  a.tabsize = w.sp.tabsize;
  a.G = w.sp.G;
  a.tag = w.tag;
  a.dx = dx;
  a.dy = dy;
  a.tplain = w.tplain;
  a.tbody = w.tbody;
  a.tslot = w.tslot;
  a.part = w.part;
  a.bpart = w.bpart;
  a.nb = nb;
  const double hx = grid_hx(g), hy = grid_hy(g);
  const double rr = hy / hx, qq = hx / hy;
  a.cC = (T)(4.0 / 3.0 * (rr + qq));
  a.cE = (T)(-2.0 / 3.0 * rr + qq / 3.0);
  a.cN = (T)(-2.0 / 3.0 * qq + rr / 3.0);
  a.cD = (T)(-(rr + qq) / 6.0);
  a.ry = (T)rr;
  if (w.cellcoef) {
    // element entries from a per-cell table: the product has no geometry to rebuild
    if constexpr (sizeof(T) == sizeof(double))
      a.kcoef = reinterpret_cast<const T*>(w.kc64);
    else
      a.kcoef = reinterpret_cast<const T*>(w.kc32);
    a.tgeo = w.tgeo;
  }
  return a;
}

// Stored element entries for the geometry tasks (Schedule::kst): slabs numbered in
// task order, each cell's K_e by the 2x2 Gauss rule from the FP64 displacements,
// kept in the precision of the iteration.
template <typename T>
static void launch_elem_coef(const SolveWs& w, double ry, T* kc, hipStream_t st) {
  const int nb = (w.L.ntasks() + WAVES - 1) / WAVES;
  if (w.L.hc == 8)
    k_elem_coef<T, 8><<<nb, BLOCK, 0, st>>>(w.L, ry, w.tag, w.dx, w.dy, w.tgeo, kc);
  else if (w.L.hc == 5)
    k_elem_coef<T, 5><<<nb, BLOCK, 0, st>>>(w.L, ry, w.tag, w.dx, w.dy, w.tgeo, kc);
  else
    k_elem_coef<T, 4><<<nb, BLOCK, 0, st>>>(w.L, ry, w.tag, w.dx, w.dy, w.tgeo, kc);
}

template <typename T>
static void launch_cells_to_slab(const SolveWs& w, T* kc, hipStream_t st) {
  const int nb = (w.L.ntasks() + WAVES - 1) / WAVES;
  if (w.L.hc == 8)
    k_cells_to_slab<T, 8><<<nb, BLOCK, 0, st>>>(w.L, w.cellcoef, w.tgeo, kc);
  else if (w.L.hc == 5)
    k_cells_to_slab<T, 5><<<nb, BLOCK, 0, st>>>(w.L, w.cellcoef, w.tgeo, kc);
  else
    k_cells_to_slab<T, 4><<<nb, BLOCK, 0, st>>>(w.L, w.cellcoef, w.tgeo, kc);
}

static int element_entries(const mfp_grid& g, const SolveWs& w, hipStream_t st) {
  k_assign_geo<<<1, 256, 0, st>>>(w.L.ntasks(), w.tplain, w.tgeo, w.ngeo);
  if (w.cellcoef) {
    if (w.kc64) launch_cells_to_slab<double>(w, w.kc64, st);
    if (w.kc32) launch_cells_to_slab<float>(w, w.kc32, st);
    MFP_TRY_HIP(hipGetLastError());
    return MFP_OK;
  }
  const double ry = grid_hy(g) / grid_hx(g);
  if (w.kc64) launch_elem_coef<double>(w, ry, w.kc64, st);
  if (w.kc32) launch_elem_coef<float>(w, ry, w.kc32, st);
  MFP_TRY_HIP(hipGetLastError());
  return MFP_OK;
}

// Common setup: tags, scaled displacements, lifting, tile metadata.
static int setup(const mfp_grid& g, const mfp_circle* circles_h, int nb, const double* disp,
                 const int8_t* body, const mfp_flow* flow, int precision, const SolveWs& w,
                 hipStream_t st, const mfp_circle* bc_circle = nullptr) {
  SetupArgs s{};
  s.L = w.L;
  s.nx = g.nx;
  s.ny = g.ny;
  s.x0 = g.x0;
  s.y0 = g.y0;
  s.hx = grid_hx(g);
  s.hy = grid_hy(g);
  s.inv_hx = 1.0 / s.hx;
  s.U = flow ? flow->U : 0.0;
  for (int k = 0; k < 4; ++k) s.bc[k] = flow ? flow->side_bc[k] : MFP_BC_NATURAL;
  // circle 0 for the isolated-cylinder boundary data (the potential passes it alone)
  const mfp_circle* c0 = bc_circle ? bc_circle : (nb > 0 ? circles_h : nullptr);
  if (c0) {
    s.c0x = c0->cx;
    s.c0y = c0->cy;
    s.c0r = c0->r;
  }
  s.disp = disp;
  s.body = body;
  s.tag = w.tag;
  s.dx = w.dx;
  s.dy = w.dy;
  s.dxf = precision != MFP_FP64 ? w.dxf : nullptr;
  s.dyf = precision != MFP_FP64 ? w.dyf : nullptr;
  s.g = w.g;
  s.x = w.x;
  s.r = w.r;
  s.p0 = w.p0;
  s.p1 = w.p1;
  s.q = w.q;
  s.nfree = w.nfree;
  s.phi = w.phi;
  s.fixed_mask = w.fixed_mask;
  for (int b = 0; b < MFP_MAX_BODIES; ++b) s.fixed[b] = w.fixed[b];
  if (w.L.nstrip > SEG_MAX_STRIPS || w.L.nchunk > 0xffff ||
      (unsigned long long)w.L.n * sizeof(double) >= (1ull << 32)) {
    set_error("grid too large (nx <= %d, ny <= %d, padded nodes < 2^29)",
              SEG_MAX_STRIPS * SW - 1, 0xffff * 4 - 1);
    return MFP_E_ARG;
  }
  MFP_TRY_HIP(hipMemsetAsync(w.st, 0, sizeof(DevState), st));
  MFP_TRY_HIP(hipMemsetAsync(w.st2, 0, sizeof(DevState), st));
  if (precision != MFP_FP64) {
    // every padded entry of the FP32 vectors starts at zero (the apply writes owned
    // nodes only)
    for (float* f : {w.xf, w.rf, w.p0f, w.p1f, w.qf, w.r1f, w.q1f})
      MFP_TRY_HIP(hipMemsetAsync(f, 0, sizeof(float) * w.L.n, st));
  }
  for (double* d : {w.r1, w.q1}) MFP_TRY_HIP(hipMemsetAsync(d, 0, sizeof(double) * w.L.n, st));
  MFP_TRY_HIP(hipMemsetAsync(w.nfree, 0, sizeof(long long), st));
  k_setup<<<grid_blocks(w.L.n), BLOCK, 0, st>>>(s);
  MFP_TRY_HIP(hipGetLastError());
  k_task_meta<<<(w.L.ntasks() + WAVES - 1) / WAVES, BLOCK, 0, st>>>(w.L, w.tag, w.dx, w.dy,
                                                                     w.tplain, w.tbody);
  MFP_TRY_HIP(hipGetLastError());
  k_assign_slots<<<1, BLOCK, 0, st>>>(w.L.ntasks(), w.tbody, w.tslot, w.nslots);
  MFP_TRY_HIP(hipGetLastError());
  k_seg_plan<<<1, 1024, 0, st>>>(w.L, w.tplain, w.sp.target, WAVES * w.sp.G, w.sp.tabsize,
                                 w.segtab);
  MFP_TRY_HIP(hipGetLastError());
  if (w.sc.kst) MFP_TRY(element_entries(g, w, st));
  return MFP_OK;
}

}  // namespace mfp

using namespace mfp;

extern "C" size_t mfp_solve_workspace_size_opts(const mfp_grid* grid, int32_t nbody,
                                                const mfp_solver_opts* opts) {
  if (!grid || !opts || grid->nx < 2 || grid->ny < 2 || nbody < 0 || nbody > MFP_MAX_BODIES)
    return 0;
  Schedule sc;
  if (resolve_schedule(grid, opts->precision, opts, &sc) != MFP_OK) return 0;
  // the solve's layout, and the element apply's (4-row tasks, geometry on the fly)
  const size_t a = solve_layout(grid, nbody, opts->precision, nullptr, nullptr, &sc);
  const size_t b = solve_layout(grid, nbody, opts->precision, nullptr, nullptr);
  return a > b ? a : b;
}

extern "C" size_t mfp_solve_workspace_size(const mfp_grid* grid, int32_t nbody,
                                           int32_t precision) {
  mfp_solver_opts o{};
  o.precision = precision;
  return mfp_solve_workspace_size_opts(grid, nbody, &o);
}

extern "C" int mfp_element_apply(const mfp_grid* grid, const double* disp,
                                 const int8_t* body, int32_t precision, const void* p,
                                 void* q, int32_t repeat, double* apply_ms_h, void* ws,
                                 size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_grid(grid));
  if (!disp || !body || !p || !q || !ws || repeat < 1) {
    set_error("NULL pointer or repeat < 1");
    return MFP_E_ARG;
  }
  if (precision != MFP_FP64 && precision != MFP_FP32) {
    set_error("precision must be MFP_FP64 or MFP_FP32");
    return MFP_E_ARG;
  }
  const int nbmax = MFP_MAX_BODIES;
  const size_t need = solve_layout(grid, nbmax, precision, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveWs w;
  solve_layout(grid, nbmax, precision, ws, &w);
  const mfp_grid& g = *grid;
  MFP_TRY(setup(g, nullptr, nbmax, disp, body, nullptr, precision, w, st));
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  const size_t esz = precision == MFP_FP64 ? sizeof(double) : sizeof(float);
  void* src = precision == MFP_FP64 ? (void*)w.p0 : (void*)w.p0f;
  void* dst = precision == MFP_FP64 ? (void*)w.q : (void*)w.qf;
  // scatter p into the padded layout
  MFP_TRY_HIP(hipMemsetAsync(src, 0, esz * w.L.n, st));
  if (precision == MFP_FP64)
    k_to_padded<double><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, (const double*)p, (double*)src);
  else
    k_to_padded<float><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, (const float*)p, (float*)src);
  MFP_TRY_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  MFP_TRY_HIP(hipEventCreate(&e0));
  MFP_TRY_HIP(hipEventCreate(&e1));
  MFP_TRY_HIP(hipEventRecord(e0, st));
  for (int k = 0; k < repeat; ++k) {
    if (precision == MFP_FP64) {
      ApplyArgs<double> a = make_apply_args<double>(w, g, nbmax, w.dx, w.dy);
      a.src = w.p0;
      a.q = w.q;
      a.write_all = 1;
      launch_apply<double>(w.L.hc, w.sp.G, st, a);
    } else {
      ApplyArgs<float> a = make_apply_args<float>(w, g, nbmax, w.dxf, w.dyf);
      a.src = w.p0f;
      a.q = w.qf;
      a.write_all = 1;
      launch_apply<float>(w.L.hc, w.sp.G, st, a);
    }
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      set_error("apply launch: %s", hipGetErrorString(le));
      return MFP_E_HIP;
    }
  }
  MFP_TRY_HIP(hipEventRecord(e1, st));
  if (precision == MFP_FP64)
    k_from_padded<double><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, (const double*)dst, (double*)q);
  else
    k_from_padded<float><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, (const float*)dst, (float*)q);
  MFP_TRY_HIP(hipGetLastError());
  MFP_TRY_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  MFP_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (apply_ms_h) *apply_ms_h = ms / repeat;
  return MFP_OK;
}

struct CgCount {
  long long iters = 0;     // index of the launch that stopped the last run
  long long applies = 0;   // operator applications over all runs
  double tsum = 0.0;       // sampled kernel durations (ms)
  long long tcnt = 0;
  int blocks = 0;          // launch shape of the last run: blocks, wavefronts per block,
  int block_waves = 0;     // element mode (1 geometry on the fly, 2 stored entries)
  int element_mode = 0;
};

// The one-kernel iteration over one set of vectors (FP64: w.r/r1, p0/p1, q/q1, x;
// FP32: the float copies and the correction e in xf): the fixed kernel arguments and
// both parity slots of every double-buffered array; at(j) gives launch j's arguments.
template <typename T>
struct StepRun {
  StepArgs<T> a;
  T* r[2];
  T* p[2];
  T* q[2];
  double* part[2];
  double* bpart[2];
  StepArgs<T> at(long long j) const {
    StepArgs<T> b = a;
    const int c = (int)(j & 1), pv = c ^ 1;
    b.j = j;
    b.rp = r[pv];
    b.qp = q[pv];
    b.pp = p[pv];
    b.rc = r[c];
    b.qc = q[c];
    b.pc = p[c];
    b.part_p = part[pv];
    b.part_c = part[c];
    b.bpart_p = bpart[pv];
    b.bpart_c = bpart[c];
    return b;
  }
};

template <typename T>
static StepRun<T> make_step_run(const SolveWs& w, const mfp_grid& g, int nb, const T* dx,
                                const T* dy, T* r0, T* r1, T* p0, T* p1, T* q0, T* q1, T* x,
                                DevState* st) {
  StepRun<T> s{};
  StepArgs<T>& a = s.a;
  a.P = w.L.P;
  a.nstrip = w.L.nstrip;
  a.nchunk = w.L.nchunk;
  a.tplain = w.tplain;
  a.tag = w.tag;
  a.dx = dx;
  a.dy = dy;
  a.tbody = w.tbody;
  a.tslot = w.tslot;
  a.nslots = w.nslots_h;
  a.x = x;
  a.st = st;
  a.nb = nb;
  // Streaming stores once the iteration's seven vectors clearly exceed the 256 MiB
  // memory-side cache of the target (measured: 478 MB faster streaming, 239 MB faster
  // cached), and also while they fit in the 8 x 4 MiB of L2: cached lines are then
  // still dirty when the launch ends and are written back in its tail, where streamed
  // ones left during it (measured at 29 MB: 14.1 -> 13.8 us per iteration; at 59 and
  // 118 MB cached stores are 13% and 15% faster).
  const double vbytes = 7.0 * (double)w.L.n * sizeof(T);
  a.stream = (vbytes > 320.0 * 1024 * 1024 || vbytes <= 32.0 * 1024 * 1024) ? 1 : 0;
  if (w.sc.stream >= 0) a.stream = w.sc.stream;
  // stored element entries of this precision, if the schedule keeps them
  const T* kc = nullptr;
  if constexpr (sizeof(T) == sizeof(double))
    kc = reinterpret_cast<const T*>(w.kc64);
  else
    kc = reinterpret_cast<const T*>(w.kc32);
  if (w.sc.kst && kc) {
    a.kcoef = kc;
    a.tgeo = w.tgeo;
  }
  const double hx = grid_hx(g), hy = grid_hy(g);
  const double rr = hy / hx, qq = hx / hy;
  a.cC = (T)(4.0 / 3.0 * (rr + qq));
  a.cE = (T)(-2.0 / 3.0 * rr + qq / 3.0);
  a.cN = (T)(-2.0 / 3.0 * qq + rr / 3.0);
  a.cD = (T)(-(rr + qq) / 6.0);
  a.ry = (T)rr;
  s.r[0] = r0;
  s.r[1] = r1;
  s.p[0] = p0;
  s.p[1] = p1;
  s.q[0] = q0;
  s.q[1] = q1;
  s.part[0] = w.spart;
  s.part[1] = w.spart + 4 * GMAX;
  s.bpart[0] = w.bpart;
  s.bpart[1] = w.bpart + w.bstride;
  return s;
}

// Start of a run at launch k0 (state of slot (k0-1)&1): the residual slot takes the
// FP64 residual w.r (converted for FP32) with its partials, the body state comes from
// the outer (FP64) state.  fresh: no previous direction; correction: the iterate is a
// correction that starts at zero (inner FP32 solve); stop_rel > 0: threshold relative
// to the start residual; kmax_abs: last launch index.
template <typename T>
static int step_start(const SolveWs& w, int nb, const StepRun<T>& a, long long k0, bool fresh,
                      bool correction, double stop_rel, long long kmax_abs, hipStream_t st,
                      int* npart0) {
  const int slot = (int)((k0 + 1) & 1);
  const int G2 = loop_blocks(w.L.n);
  k_step_start<T><<<G2, BLOCK, 0, st>>>(w.L.n, w.r, a.r[slot], a.part[slot]);
  k_step_bodies<<<1, 64, 0, st>>>(w.st, a.a.st, nb, slot, fresh ? 1 : 0, correction ? 1 : 0,
                                  stop_rel, kmax_abs);
  MFP_TRY_HIP(hipGetLastError());
  *npart0 = G2;
  return MFP_OK;
}

// Host-visible copy of a solve's outcome: DevState from `iters` through `done`
// (iters, kmax, outer_count, done), copied in one piece.
// Host-visible copy of a solve's outcome: DevState from `iters` through `done`
// (iters, kmax, outer_count, done), copied in one piece.
struct OutcomeCopy {
  long long iters, kmax, outer_count;
  int done, pad_;
};
static_assert(offsetof(DevState, done) - offsetof(DevState, iters) ==
                  offsetof(OutcomeCopy, done) - offsetof(OutcomeCopy, iters),
              "DevState outcome fields must match OutcomeCopy");

// Pinned host memory of a host thread's solves, allocated on first use and kept for
// the life of the process: the stop code that the stopping launch writes (the host
// polls it) and the outcome copy read at the end of a run.
struct HostIo {
  OutcomeCopy out;
  int flag;
};
static HostIo* host_io(int** flag_dev) {
  static thread_local HostIo* io = nullptr;
  static thread_local int* dflag = nullptr;
  if (!io) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(HostIo), hipHostMallocDefault) != hipSuccess) return nullptr;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, &static_cast<HostIo*>(p)->flag, 0) != hipSuccess) {
      (void)hipHostFree(p);
      return nullptr;
    }
    io = static_cast<HostIo*>(p);
    dflag = static_cast<int*>(d);
  }
  *flag_dev = dflag;
  return io;
}

// Host loop of the one-kernel CG from launch k0.  Launches are enqueued in batches of
// `check_every` (0 -> 16), each followed by an event.  The stopping launch writes its
// stop code into pinned host memory as well; the host looks at it after a batch's
// event has completed, and only once the next batch is enqueued, so the device never
// drains between batches and no copy runs between them.  An outcome is seen at most
// one batch late; the launches still in flight then return at once.  Afterwards the
// outcome fields are copied once and the iterate takes the stopping launch's alpha p.
// With profile_every = n > 0, every n-th batch that ends before the stop is timed
// between the events that end it and the batch before it (nothing else runs on the
// stream in between), and its mean per launch enters cnt.
// Returns the done code (1 converged, 2 breakdown, 3 kmax) or a negative status;
// cnt->iters is the stopping launch.
template <typename T>
static int step_run(const SolveWs& w, StepRun<T> run, const mfp_solver_opts& o, hipStream_t st,
                    CgCount* cnt, long long k0) {
  if (w.L.hc != 4 && w.L.hc != 5 && w.L.hc != 8) {
    set_error("internal: the CG iteration kernel needs 4-, 5- or 8-row tasks");
    return MFP_E_ARG;
  }
  int* flag_dev = nullptr;
  HostIo* io = host_io(&flag_dev);
  if (!io) {
    set_error("pinned host memory for the stop flag: allocation failed");
    return MFP_E_HIP;
  }
  volatile int* flag = &io->flag;
  *flag = 0;  // no launch of an earlier run is in flight (every run ends synchronised)
  int G = step_blocks<T>(w.L, run.a.kcoef ? 1 : 0, w.sc.blocks);
  if (w.pair_blocks > 0 &&
      pair_blocks<T>(w.L.hc, w.L.ntasks(), run.a.kcoef != nullptr) == w.pair_blocks) {
    run.a.wtask = w.wtask;
    G = w.pair_blocks;
  }
  cnt->blocks = G;
  cnt->block_waves = run.a.wtask ? 8 : WAVES;
  cnt->element_mode = run.a.kcoef ? 2 : 1;
  const int every = o.check_every > 0 ? o.check_every : 16;
  const int prof = o.profile_every > 0 ? o.profile_every : 0;
  // ev[b % NE] marks the end of batch b - 1 (ev[0]: the start of batch 0); an event is
  // re-recorded three batches after it was last read
  constexpr int NE = 4;
  hipEvent_t ev[NE];
  int created = 0;
  int status = MFP_OK;
  for (int i = 0; i < NE && status == MFP_OK; ++i) {
    if (hipEventCreateWithFlags(&ev[i], prof ? hipEventDefault : hipEventDisableTiming) !=
        hipSuccess)
      status = MFP_E_HIP;
    else
      ++created;
  }
  long long j = k0;
  run.a.k0 = k0;
  run.a.host_done = flag_dev;
  const long long guard =
      (o.kmax > 2000 + 2 * k0 ? o.kmax : 2000 + 2 * k0) + 2LL * every + 2;
  long long b = 0;  // batch being enqueued
  if (status == MFP_OK && hipEventRecord(ev[0], st) != hipSuccess) status = MFP_E_HIP;
  while (status == MFP_OK) {
    for (int m = 0; m < every; ++m, ++j) launch_step<T>(G, st, run.at(j), w.L.hc);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) le = hipEventRecord(ev[(b + 1) % NE], st);
    if (le == hipSuccess && b > 0) le = hipEventSynchronize(ev[b % NE]);  // batch b - 1
    if (le != hipSuccess) {
      set_error("CG loop: %s", hipGetErrorString(le));
      status = MFP_E_HIP;
      break;
    }
    if (b > 0) {
      if (*flag != 0) break;  // batch b - 1 held the stopping launch
      if (prof && (b - 1) % prof == 0) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[(b - 1) % NE], ev[b % NE]) == hipSuccess) {
          cnt->tsum += ms;
          cnt->tcnt += every;
        }
      }
      // every run stops by its iteration cap; should the flag never show, the device
      // state decides after the loop
      if (j - k0 > guard) break;
    }
    ++b;
  }
  // the batch still in flight (launches that return at once) ends, then the outcome
  hipError_t le = hipSuccess;
  if (status == MFP_OK) le = hipEventSynchronize(ev[(b + 1) % NE]);
  if (status == MFP_OK && le == hipSuccess)
    le = hipMemcpyAsync(&io->out, reinterpret_cast<const char*>(run.a.st) + offsetof(DevState, iters),
                        offsetof(DevState, done) + sizeof(int) - offsetof(DevState, iters),
                        hipMemcpyDeviceToHost, st);
  if (status == MFP_OK && le == hipSuccess) le = hipStreamSynchronize(st);
  if (status == MFP_OK && le != hipSuccess) {
    set_error("CG loop: %s", hipGetErrorString(le));
    status = MFP_E_HIP;
  }
  const OutcomeCopy outcome = io->out;
  for (int i = 0; i < created; ++i) (void)hipEventDestroy(ev[i]);
  if (status != MFP_OK) return status;
  if (outcome.done == 0) {
    set_error("internal: CG loop ended without an outcome");
    return MFP_E_HIP;
  }
  k_finish<T><<<loop_blocks(w.L.n), BLOCK, 0, st>>>(w.L.n, run.a.x, run.p[0], run.p[1], run.a.st);
  MFP_TRY_HIP(hipGetLastError());
  cnt->iters = outcome.iters;
  cnt->applies += outcome.iters - k0;
  return outcome.done;
}

// b - A x in FP64 from the current iterate: w = g + T x, q = K w, r = -T^T q, then
// k_resid_finalize in the given mode.
static int residual64(const mfp_grid& g, int nb, const SolveWs& w, hipStream_t st, int mode,
                      double rtol, double stop_abs = 0.0) {
  const int G2 = loop_blocks(w.L.n);
  k_form_w<double><<<G2, BLOCK, 0, st>>>(w.L.n, w.tag, w.x, w.g, w.st, w.p0);
  ApplyArgs<double> a = make_apply_args<double>(w, g, nb, w.dx, w.dy);
  a.src = w.p0;
  a.q = w.q;
  launch_apply<double>(w.L.hc, w.sp.G, st, a);
  k_resid<<<G2, BLOCK, 0, st>>>(w.L.n, w.q, w.r, w.part2, mode != 1 ? 1 : 0);
  k_resid_finalize<<<1, BLOCK, 0, st>>>(w.part2, G2, w.bpart, w.nslots, w.st, nb, mode,
                                        rtol * rtol, stop_abs);
  MFP_TRY_HIP(hipGetLastError());
  if (mode == 0) MFP_TRY_HIP(hipMemsetAsync(w.p0, 0, sizeof(double) * w.L.n, st));
  return MFP_OK;
}

static int read_rr(const SolveWs& w, hipStream_t st, double* rr, double* rr0) {
  double v[2];
  MFP_TRY_HIP(hipMemcpyAsync(&v[0], &w.st->rr_true, sizeof(double), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipMemcpyAsync(&v[1], &w.st->rr0, sizeof(double), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  *rr = v[0];
  *rr0 = v[1];
  return MFP_OK;
}

// FP64 CG from the state that residual64 (mode 0) prepared: one run from launch 1.
static int solve64(const mfp_grid& g, int nb, const SolveWs& w, const mfp_solver_opts& o,
                   hipStream_t st, CgCount* cnt, long long kmax = 0) {
  StepRun<double> a = make_step_run<double>(w, g, nb, w.dx, w.dy, w.r, w.r1, w.p0, w.p1,
                                              w.q, w.q1, w.x, w.st);
  a.a.hist = w.hist;
  a.a.hist_cap = HIST_CAP;
  const long long km = kmax > 0 ? kmax : o.kmax;
  MFP_TRY(step_start<double>(w, nb, a, 1, true, false, 0.0, 1 + km, st, &a.a.npart0));
  return step_run<double>(w, a, o, st, cnt, 1);
}

// Mixed precision.  FP32 CG (FP32 vectors and element apply, FP64 scalars and body
// sums) on the correction e, started from r32 = r64 = b - A x.  Each time the FP32
// residual norm has dropped by `delta` since the last FP64 residual, x += e in FP64,
// e = 0, the residual is recomputed with the FP64 apply and replaces r32, and the
// iteration restarts with its current direction (beta from the new residual).
// MFP_FP32 runs one run to rtol and reports the FP64 residual.  Returns the final done
// code (0: FP32 stagnation, continue in FP64).
static long long k0_cap(long long k) { return 2 * k > 2000 ? 2 * k : 2000; }

static int solve_mixed(const mfp_grid& g, int nb, const SolveWs& w, const mfp_solver_opts& o,
                       hipStream_t st, CgCount* cnt, long long* total_iters, long long* updates,
                       bool* stagnated) {
  const bool ir = o.precision == MFP_FP32_IR;
  const double delta = ir ? (o.inner_rtol > 0 && o.inner_rtol < 1 ? o.inner_rtol : 0.1) : o.rtol;
  const int max_upd = o.max_outer > 0 ? o.max_outer : 1000;
  const int G2 = loop_blocks(w.L.n);
  double rr = 0, rr0 = 0;
  MFP_TRY(read_rr(w, st, &rr, &rr0));
  if (rr <= o.rtol * o.rtol * rr0) return 1;
  MFP_TRY_HIP(hipMemsetAsync(w.xf, 0, sizeof(float) * w.L.n, st));
  StepRun<float> a = make_step_run<float>(w, g, nb, w.dxf, w.dyf, w.rf, w.r1f, w.p0f, w.p1f,
                                            w.qf, w.q1f, w.xf, w.st2);
  a.a.hist = w.hist;
  a.a.hist_cap = HIST_CAP;
  long long k0 = 1;
  bool fresh = true;
  int code = 0;
  while (true) {
    // a run may take at most max(2000, 2 x all iterations so far); one that does not
    // reach its reduction within that is taken as FP32 stagnation
    const long long cap = ir ? k0_cap(k0 - 1) : o.kmax;
    long long kabs = k0 + cap;
    if (kabs > 1 + o.kmax) kabs = 1 + o.kmax;
    MFP_TRY(step_start<float>(w, nb, a, k0, fresh, true, delta * delta, kabs, st, &a.a.npart0));
    code = step_run<float>(w, a, o, st, cnt, k0);
    if (code < 0) return code;
    const long long J = cnt->iters;
    *total_iters = J - 1;
    // fold the correction into the FP64 iterate and recompute the true residual
    k_ir_update<<<G2, BLOCK, 0, st>>>(w.L.n, w.x, w.xf, w.st, w.st2, nb, (int)(J & 1));
    MFP_TRY_HIP(hipGetLastError());
    MFP_TRY(residual64(g, nb, w, st, 2, o.rtol));
    cnt->applies += 1;
    ++*updates;
    MFP_TRY(read_rr(w, st, &rr, &rr0));
    if (rr <= o.rtol * o.rtol * rr0) return 1;
    if (!ir) return code == 2 ? 2 : 3;
    if (code == 3 && J - 1 >= o.kmax) return 3;
    if (code != 1 || *updates >= max_upd) {
      *stagnated = true;
      return 0;
    }
    fresh = false;
    k0 = J;
  }
}

// Warm start: body unknowns from the first node (row-major) of each body in psi0.
__global__ void k_warm_xb(int nx, int ny, int nb, const int* __restrict__ boxes,
                          const int8_t* __restrict__ body, const double* __restrict__ psi0,
                          DevState* st) {
  const int b = threadIdx.x;
  if (b >= nb) return;
  const int i0 = boxes[4 * b], i1 = boxes[4 * b + 1], j0 = boxes[4 * b + 2], j1 = boxes[4 * b + 3];
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      const long long n = (long long)j * (nx + 1) + i;
      if (body[n] == b) {
        st->xb[0][b] = psi0[n];
        return;
      }
    }
}

// x = psi0 at free nodes (padded layout).
__global__ void k_warm_x(Layout L, int nx, int ny, const int8_t* __restrict__ tag,
                         const double* __restrict__ psi0, double* __restrict__ x) {
  const long long nn = (long long)(nx + 1) * (ny + 1);
  for (long long nd = blockIdx.x * (long long)blockDim.x + threadIdx.x; nd < nn;
       nd += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(nd / (nx + 1)), i = (int)(nd - (long long)j * (nx + 1));
    const long long e = node_index(L, i, j);
    if (tag_own(tag[e])) x[e] = psi0[nd];
  }
}

struct SolveInfo {
  int done = 0;
  bool stagnated = false;
  long long iters = 0, inner = 0, outer = 0, applies = 0, apply_samples = 0;
  double apply_ms = 0.0, solve_ms = 0.0;
  double kappa = 0.0, ritz_min = 0.0, ritz_max = 0.0;
  long long kappa_steps = 0;
  int step_blocks = 0, step_block_waves = 0, step_element_mode = 0;
};

// Number of eigenvalues below x of the symmetric tridiagonal with diagonal d[0..m) and
// squared off-diagonals e2[1..m) (e2[k] couples k-1 and k): the sign changes of the
// Sturm sequence of leading-minor ratios.
static int sturm_count(const std::vector<double>& d, const std::vector<double>& e2, double x,
                       double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  for (size_t k = 0;;) {
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    if (++k >= d.size()) break;
    q = (d[k] - x) - e2[k] / q;
  }
  return cnt;
}

// Condition estimate from the CG scalars of one run (section "Matrix-Free Conjugate
// Gradient..." / Algorithm 1: alpha = r.r / p.Ap, beta = r_new.r_new / r.r).  CG on A
// is the Lanczos process on A started from the first residual; its tridiagonal T has
//   T_11 = 1/alpha_1,  T_kk = 1/alpha_k + beta_k/alpha_(k-1),
//   T_k,k-1 = sqrt(beta_k)/alpha_(k-1)
// (alpha_k: step along p_k; beta_k: p_k = r_k + beta_k p_(k-1)).  hist holds launch j's
// (alpha_(j-1), beta_j) at [2j], [2j+1] for j = 1..J (2J + 2 entries); J is the last
// launch kept, so T has order J-1, cut at the first step length that is not positive
// and finite.  Extreme eigenvalues by bisection from the Gershgorin interval.
static void lanczos_kappa(const std::vector<double>& hist, long long J, SolveInfo* info) {
  const long long m = J - 1;
  if ((long long)hist.size() < 2 * (J + 1)) return;
  std::vector<double> d, e2;
  for (long long k = 1; k <= m; ++k) {
    const double ak = hist[2 * (k + 1)];  // alpha_k, formed by launch k+1
    if (!(ak > 0.0) || !std::isfinite(ak)) break;
    if (k == 1) {
      d.push_back(1.0 / ak);
      e2.push_back(0.0);
    } else {
      const double ap = hist[2 * k], bk = hist[2 * k + 1];  // alpha_(k-1), beta_k
      if (!(bk >= 0.0) || !std::isfinite(bk)) break;
      d.push_back(1.0 / ak + bk / ap);
      e2.push_back(bk / (ap * ap));
    }
  }
  const size_t n = d.size();
  if (n < 2) return;
  double lo = d[0], hi = d[0], emax = 0.0;
  for (size_t k = 0; k < n; ++k) {
    const double r = (k > 0 ? std::sqrt(e2[k]) : 0.0) + (k + 1 < n ? std::sqrt(e2[k + 1]) : 0.0);
    lo = std::fmin(lo, d[k] - r);
    hi = std::fmax(hi, d[k] + r);
    emax = std::fmax(emax, e2[k]);
  }
  const double pivmin = 1e-300 * std::fmax(1.0, emax);
  const double span = hi - lo;
  lo -= 1e-12 * span;
  hi += 1e-12 * span;
  // smallest: count(x) >= 1 iff x > lambda_min; largest: count(x) == n iff x > lambda_max
  double a = lo, b = hi;
  for (int it = 0; it < 200 && b - a > 1e-13 * std::fabs(b); ++it) {
    const double c = 0.5 * (a + b);
    (sturm_count(d, e2, c, pivmin) >= 1 ? b : a) = c;
  }
  const double lmin = 0.5 * (a + b);
  a = lo;
  b = hi;
  for (int it = 0; it < 200 && b - a > 1e-13 * std::fabs(b); ++it) {
    const double c = 0.5 * (a + b);
    (sturm_count(d, e2, c, pivmin) >= (int)n ? b : a) = c;
  }
  const double lmax = 0.5 * (a + b);
  info->ritz_min = lmin;
  info->ritz_max = lmax;
  info->kappa = lmin > 0.0 ? lmax / lmin : 0.0;
  info->kappa_steps = (long long)n;
}

static int check_solve_args(const mfp_grid* grid, const mfp_circle* circles_h, int nbody,
                            const double* disp, const int8_t* kind, const int8_t* body,
                            const mfp_flow* flow, const mfp_solver_opts* opts, const void* ws) {
  MFP_TRY(check_geometry(grid, circles_h, nbody));
  if (!disp || !kind || !body || !flow || !opts || !ws) {
    set_error("NULL argument");
    return MFP_E_ARG;
  }
  for (int k = 0; k < 4; ++k)
    if (flow->side_bc[k] < MFP_BC_NATURAL || flow->side_bc[k] > MFP_BC_DIRICHLET_CYLPHI) {
      set_error("invalid side boundary code");
      return MFP_E_ARG;
    }
  if (!std::isfinite(flow->U)) {
    set_error("U is not finite");
    return MFP_E_ARG;
  }
  if (opts->precision < MFP_FP64 || opts->precision > MFP_FP32_IR) {
    set_error("unknown precision %d", opts->precision);
    return MFP_E_ARG;
  }
  if (!(opts->rtol > 0.0) || opts->kmax < 1) {
    set_error("rtol must be > 0 and kmax >= 1");
    return MFP_E_ARG;
  }
  return MFP_OK;
}

static void circle_boxes(const mfp_grid& g, const mfp_circle* c, int nb, int* boxes) {
  for (int b = 0; b < nb; ++b) {
    const Box bx = circle_box(g, c[b], 1, 0, g.nx - 1, 0, g.ny - 1);
    boxes[4 * b] = bx.i0;
    boxes[4 * b + 1] = bx.i1;
    boxes[4 * b + 2] = bx.j0;
    boxes[4 * b + 3] = bx.j1;
  }
}

// Setup, CG (FP64, or FP32 with FP64 refinement and FP64 fallback), true residual.
// bb_h: extra right-hand side of the body rows (NULL: none); zero_g: homogeneous
// Dirichlet data (adjoint).
static int solve_core(const mfp_grid& g, const mfp_circle* circles_h, int nb, const double* disp,
                      const int8_t* body, const mfp_flow* flow, const mfp_solver_opts* opts,
                      const double* bb_h, bool zero_g, const SolveWs& w, hipStream_t st,
                      SolveInfo* info, const mfp_circle* bc_circle = nullptr) {
  MFP_TRY(setup(g, circles_h, nb, disp, body, flow, opts->precision, w, st, bc_circle));
  if (zero_g) MFP_TRY_HIP(hipMemsetAsync(w.g, 0, sizeof(double) * w.L.n, st));
  if (bb_h && nb > 0)
    MFP_TRY_HIP(hipMemcpyAsync(w.st->bb, bb_h, sizeof(double) * nb, hipMemcpyHostToDevice, st));
  long long kmax = opts->kmax;
  MFP_TRY_HIP(hipMemcpyAsync(&w.st->kmax, &kmax, sizeof(long long), hipMemcpyHostToDevice, st));
  if (nb > 0) {
    int boxes[4 * MFP_MAX_BODIES];
    circle_boxes(g, circles_h, nb, boxes);
    MFP_TRY_HIP(hipMemcpyAsync(w.boxes, boxes, sizeof(int) * 4 * nb, hipMemcpyHostToDevice, st));
    MFP_TRY_HIP(hipMemcpyAsync(w.circ, circles_h, sizeof(mfp_circle) * nb,
                               hipMemcpyHostToDevice, st));
  }
  MFP_TRY_HIP(hipMemcpyAsync(&w.nslots_h, w.nslots, sizeof(int), hipMemcpyDeviceToHost, st));
  // one task per wavefront when the tasks fit (not with stored entries or a forced
  // launch size)
  w.pair_blocks = 0;
  int pcus = 0;
  if (w.sc.blocks == 0) {
    const bool kst = w.sc.kst != 0;
    pcus = pair_blocks<double>(w.L.hc, w.L.ntasks(), kst);
    if (opts->precision != MFP_FP64 && !pcus) pcus = pair_blocks<float>(w.L.hc, w.L.ntasks(), kst);
  }
  const size_t ntp = pcus ? (size_t)w.L.ntasks() : 0;
  std::vector<uint8_t> plain(ntp);
  std::vector<unsigned long long> tbody(ntp);
  std::vector<int> tslot(ntp), tgeo(w.sc.kst ? ntp : 0);
  if (pcus) {
    MFP_TRY_HIP(hipMemcpyAsync(plain.data(), w.tplain, ntp, hipMemcpyDeviceToHost, st));
    MFP_TRY_HIP(hipMemcpyAsync(tbody.data(), w.tbody, sizeof(unsigned long long) * ntp,
                               hipMemcpyDeviceToHost, st));
    MFP_TRY_HIP(hipMemcpyAsync(tslot.data(), w.tslot, sizeof(int) * ntp, hipMemcpyDeviceToHost, st));
    if (!tgeo.empty())
      MFP_TRY_HIP(hipMemcpyAsync(tgeo.data(), w.tgeo, sizeof(int) * ntp, hipMemcpyDeviceToHost, st));
  }
  MFP_TRY_HIP(hipStreamSynchronize(st));  // host-side staging buffers above, slot count
  if (pcus) {
    std::vector<int2> tab(8 * (size_t)pcus);
    if (pair_table(plain.data(), tbody.data(), tslot.data(), tgeo.empty() ? nullptr : tgeo.data(),
                   w.L.ntasks(), pcus, tab.data())) {
      MFP_TRY_HIP(hipMemcpyAsync(w.wtask, tab.data(), sizeof(int2) * tab.size(),
                                 hipMemcpyHostToDevice, st));
      MFP_TRY_HIP(hipStreamSynchronize(st));  // the table's staging buffer
      w.pair_blocks = pcus;
    }
  }

  hipEvent_t e0, e1;
  MFP_TRY_HIP(hipEventCreate(&e0));
  MFP_TRY_HIP(hipEventCreate(&e1));
  MFP_TRY_HIP(hipEventRecord(e0, st));
  CgCount cnt;
  long long outer = 0, total_iters = 0;
  int done = 1;
  bool stagnated = false;
  // rtol is relative to ||b||, the residual of the zero iterate, which the first call
  // records; a warm start then replaces the iterate and the state is formed again
  // from its residual (the threshold stays rtol ||b||).  With rtol_from_start the
  // warm start's residual is the first one recorded, and the reference.
  if (!opts->psi0 || !opts->rtol_from_start) {
    MFP_TRY(residual64(g, nb, w, st, 0, opts->rtol));
    cnt.applies += 1;
  }
  if (opts->psi0) {
    const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
    k_warm_x<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, opts->psi0, w.x);
    if (nb > 0) k_warm_xb<<<1, 64, 0, st>>>(g.nx, g.ny, nb, w.boxes, body, opts->psi0, w.st);
    MFP_TRY_HIP(hipGetLastError());
    MFP_TRY(residual64(g, nb, w, st, 0, opts->rtol));
    cnt.applies += 1;
  }
  long long inner = 0;
  if (opts->precision == MFP_FP64) {
    done = solve64(g, nb, w, *opts, st, &cnt);
    if (done < 0) return done;
    total_iters = cnt.iters - 1;
  } else {
    double rr = 0, rr0 = 0;
    done = solve_mixed(g, nb, w, *opts, st, &cnt, &total_iters, &outer, &stagnated);
    if (done < 0) return done;
    inner = total_iters;
    if (opts->precision == MFP_FP32_IR && done == 0) {
      // FP64 CG from the current iterate to the original target
      stagnated = true;
      MFP_TRY(read_rr(w, st, &rr, &rr0));
      MFP_TRY(residual64(g, nb, w, st, 0, opts->rtol, opts->rtol * opts->rtol * rr0));
      cnt.applies += 1;
      long long left = opts->kmax - total_iters;
      if (left < 1) left = 1;
      done = solve64(g, nb, w, *opts, st, &cnt, left);
      if (done < 0) return done;
      total_iters += cnt.iters - 1;
    }
  }
  MFP_TRY_HIP(hipEventRecord(e1, st));
  MFP_TRY(residual64(g, nb, w, st, 1, opts->rtol));
  cnt.applies += 1;
  MFP_TRY_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (opts->estimate_kappa && cnt.iters > 2) {
    // launches 1..J hold their scalars at [2j], [2j+1] (those below HIST_CAP)
    const long long J = cnt.iters < HIST_CAP - 1 ? cnt.iters : HIST_CAP - 1;
    std::vector<double> hist(2 * (size_t)(J + 1));
    MFP_TRY_HIP(hipMemcpyAsync(hist.data(), w.hist, sizeof(double) * hist.size(),
                               hipMemcpyDeviceToHost, st));
    MFP_TRY_HIP(hipStreamSynchronize(st));
    lanczos_kappa(hist, J, info);
  }
  info->done = done;
  info->stagnated = stagnated;
  info->iters = total_iters;
  info->inner = inner;
  info->outer = outer;
  info->applies = cnt.applies;
  info->apply_ms = cnt.tcnt ? cnt.tsum / cnt.tcnt : 0.0;
  info->apply_samples = cnt.tcnt;
  info->step_blocks = cnt.blocks;
  info->step_block_waves = cnt.block_waves;
  info->step_element_mode = cnt.element_mode;
  info->solve_ms = ms;
  return MFP_OK;
}

static int finish_status(const SolveInfo& info) {
  if (info.done == 2) {
    set_error("CG breakdown (p.Ap <= 0 or non-finite)");
    return MFP_E_BREAKDOWN;
  }
  if (info.done == 3 || info.done == 0) {
    set_error("kmax or the refinement cap reached before the tolerance");
    return MFP_W_NOCONV;
  }
  if (info.stagnated) {
    set_error("FP32 refinement stagnated; finished with FP64 CG");
    return MFP_W_STAGNATION;
  }
  return MFP_OK;
}

static int fill_stats(const SolveWs& w, const SolveInfo& info, int nb, const DevState& hsd,
                      hipStream_t st, mfp_stats* stats_h) {
  if (!stats_h) return MFP_OK;
  long long nfree = 0;
  MFP_TRY_HIP(hipMemcpyAsync(&nfree, w.nfree, sizeof(long long), hipMemcpyDeviceToHost, st));
  std::vector<uint8_t> plain(w.L.ntasks());
  MFP_TRY_HIP(hipMemcpyAsync(plain.data(), w.tplain, plain.size(), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  long long nplain = 0;
  for (uint8_t v : plain) nplain += v;
  std::memset(stats_h, 0, sizeof(*stats_h));
  stats_h->iters = info.iters;
  stats_h->outer_iters = info.outer;
  stats_h->applies = info.applies;
  stats_h->n_free = nfree;
  stats_h->n_dof = nfree + nb;
  stats_h->rnorm0 = std::sqrt(hsd.rr0);
  stats_h->relres_true = hsd.rr0 > 0 ? std::sqrt(hsd.rr_true / hsd.rr0) : 0.0;
  stats_h->solve_ms = info.solve_ms;
  stats_h->apply_ms = info.apply_ms;
  stats_h->apply_samples = info.apply_samples;
  stats_h->n_tiles = w.L.ntasks();
  stats_h->n_plain_tiles = nplain;
  stats_h->inner_iters = info.inner;
  stats_h->kappa_est = info.kappa;
  stats_h->ritz_min = info.ritz_min;
  stats_h->ritz_max = info.ritz_max;
  stats_h->kappa_steps = info.kappa_steps;
  stats_h->step_blocks = info.step_blocks;
  stats_h->step_block_waves = info.step_block_waves;
  stats_h->step_element_mode = info.step_element_mode;
  return MFP_OK;
}

extern "C" int mfp_psi_solve(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                             const double* disp, const int8_t* kind, const int8_t* body,
                             const mfp_flow* flow, const mfp_solver_opts* opts,
                             int32_t pair_lo, int32_t pair_hi, double* psi, double* psi_b_h,
                             double* Q_h, double* copfi_h, double* samples,
                             int8_t* sample_body, int32_t sample_cap, int32_t* n_samples_h,
                             mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_solve_args(grid, circles_h, nbody, disp, kind, body, flow, opts, ws));
  if (!psi || (nbody > 0 && !psi_b_h)) {
    set_error("psi or psi_b_h is NULL");
    return MFP_E_ARG;
  }
  if (pair_lo >= nbody || pair_hi >= nbody) {
    set_error("pair index out of range");
    return MFP_E_ARG;
  }
  if (sample_cap < 0 || (sample_cap > 0 && (!samples || !sample_body))) {
    set_error("bad sample buffers");
    return MFP_E_ARG;
  }
  Schedule sc;
  MFP_TRY(resolve_schedule(grid, opts->precision, opts, &sc));
  const size_t need = solve_layout(grid, nbody, opts->precision, nullptr, nullptr, &sc);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveWs w;
  solve_layout(grid, nbody, opts->precision, ws, &w, &sc);
  const mfp_grid& g = *grid;
  const int nb = nbody;
  SolveInfo info;
  MFP_TRY(solve_core(g, circles_h, nb, disp, body, flow, opts, nullptr, false, w, st, &info));
  double ylo = 0, yhi = 0;
  if (pair_lo >= 0 && pair_hi >= 0) {
    ylo = circles_h[pair_lo].cy;
    yhi = circles_h[pair_hi].cy;
  }
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  k_output<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, w.x, w.g, w.st, psi,
                                               pair_lo, pair_hi, flow->U, ylo, yhi);
  MFP_TRY_HIP(hipGetLastError());
  int nsamp = 0;
  if (nb > 0) {
    SampleArgs sa{};
    sa.nx = g.nx;
    sa.ny = g.ny;
    sa.nb = nb;
    sa.x0 = g.x0;
    sa.y0 = g.y0;
    sa.hx = grid_hx(g);
    sa.hy = grid_hy(g);
    sa.hmax = sa.hx > sa.hy ? sa.hx : sa.hy;
    sa.circ = w.circ;
    sa.boxes = w.boxes;
    sa.disp = disp;
    sa.kind = kind;
    sa.body = body;
    sa.psi = psi;
    sa.st = w.st;
    sa.samples = samples;
    sa.sbody = sample_body;
    sa.cap = sample_cap;
    sa.count = w.count;
    int hb[4 * MFP_MAX_BODIES];
    circle_boxes(g, circles_h, nb, hb);
    sa.items = 0;
    for (int q = 0; q < nb; ++q) {
      sa.first[q] = sa.items;
      if (hb[4 * q + 1] >= hb[4 * q] && hb[4 * q + 3] >= hb[4 * q + 2])
        sa.items += (long long)(hb[4 * q + 1] - hb[4 * q] + 1) * (hb[4 * q + 3] - hb[4 * q + 2] + 1);
    }
    sa.first[nb] = sa.items;
    const long long nblk = (sa.items + SMP_CHUNK - 1) / SMP_CHUNK;
    if (nblk > w.sboff_n) {
      set_error("internal: too many sample cells");
      return MFP_E_ARG;
    }
    sa.boff = w.sboff;
    if (nblk > 0) {
      k_samples_count<<<(unsigned)nblk, BLOCK, 0, st>>>(sa);
      k_samples_scan<<<1, BLOCK, 0, st>>>(sa, (int)nblk);
      k_samples_write<<<(unsigned)nblk, BLOCK, 0, st>>>(sa);
    } else {
      MFP_TRY_HIP(hipMemsetAsync(w.count, 0, sizeof(int), st));
    }
    MFP_TRY_HIP(hipGetLastError());
    MFP_TRY_HIP(hipMemcpyAsync(&nsamp, w.count, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  DevState hsd;
  MFP_TRY_HIP(hipMemcpyAsync(&hsd, w.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < nb; ++b) psi_b_h[b] = hsd.xb[hsd.iters & 1][b];
  if (pair_lo >= 0 && pair_hi >= 0) {
    if (Q_h) *Q_h = hsd.Q;
    if (copfi_h) *copfi_h = hsd.copfi;
  }
  if (n_samples_h) *n_samples_h = nsamp;
  MFP_TRY(fill_stats(w, info, nb, hsd, st, stats_h));
  return finish_status(info);
}

namespace mfp {

// Schedule of a solve whose element entries come from a per-cell table: the stored
// form for every geometry task, the rest as for any solve.
static int cells_schedule(const mfp_grid* grid, const mfp_solver_opts* opts, Schedule* sc) {
  MFP_TRY(resolve_schedule(grid, opts ? opts->precision : MFP_FP64, opts, sc));
  sc->kst = 1;
  sc->cells = 1;
  return MFP_OK;
}

size_t psi_solve_cells_workspace(const mfp_grid* grid, int nbody, const mfp_solver_opts* opts) {
  Schedule sc;
  if (cells_schedule(grid, opts, &sc) != MFP_OK) return 0;
  return solve_layout(grid, nbody, opts ? opts->precision : MFP_FP64, nullptr, nullptr, &sc);
}

int psi_solve_cells(const mfp_grid* grid, const mfp_circle* circles_h, int nbody,
                    const double* disp, const int8_t* body, const double* cellcoef,
                    const mfp_flow* flow, const mfp_solver_opts* opts, int pair_lo,
                    int pair_hi, double* psi, double* psi_b_h, double* Q_h, double* copfi_h,
                    mfp_stats* stats_h, void* ws, size_t ws_bytes, hipStream_t st) {
  MFP_TRY(check_solve_args(grid, circles_h, nbody, disp, body, body, flow, opts, ws));
  if (!psi || !cellcoef || (nbody > 0 && !psi_b_h) || pair_lo >= nbody || pair_hi >= nbody) {
    set_error("NULL argument or pair index out of range");
    return MFP_E_ARG;
  }
  Schedule sc;
  MFP_TRY(cells_schedule(grid, opts, &sc));
  const size_t need = solve_layout(grid, nbody, opts->precision, nullptr, nullptr, &sc);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  SolveWs w;
  solve_layout(grid, nbody, opts->precision, ws, &w, &sc);
  w.cellcoef = cellcoef;
  const mfp_grid& g = *grid;
  SolveInfo info;
  MFP_TRY(solve_core(g, circles_h, nbody, disp, body, flow, opts, nullptr, false, w, st, &info));
  double ylo = 0, yhi = 0;
  if (pair_lo >= 0 && pair_hi >= 0) {
    ylo = circles_h[pair_lo].cy;
    yhi = circles_h[pair_hi].cy;
  }
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  k_output<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, w.x, w.g, w.st, psi,
                                               pair_lo, pair_hi, flow->U, ylo, yhi);
  MFP_TRY_HIP(hipGetLastError());
  DevState hsd;
  MFP_TRY_HIP(hipMemcpyAsync(&hsd, w.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < nbody; ++b) psi_b_h[b] = hsd.xb[hsd.iters & 1][b];
  if (pair_lo >= 0 && pair_hi >= 0) {
    if (Q_h) *Q_h = hsd.Q;
    if (copfi_h) *copfi_h = hsd.copfi;
  }
  MFP_TRY(fill_stats(w, info, nbody, hsd, st, stats_h));
  return finish_status(info);
}

}  // namespace mfp

namespace mfp {

// ---- Kutta constraints ---------------------------------------------------------------
// psi(K_b) = psi_b in place of body b's zero-circulation row.  The system stays
// linear, and with those bodies held at given values it is the constrained system
// of the other bodies: psi = S0 + sum_k c_k S_k, where S0 is the solve with every
// Kutta body held at 0 and S_k the solve without side data (U = 0) with Kutta body
// k held at 1 and the other Kutta bodies at 0.  The Kutta rows then read
// S0(K_j) + sum_k c_k S_k(K_j) = c_j, an nk x nk system solved on the host; psi_b of
// a Kutta body is c_b.

// psi += c * s over the (unpadded) nodes
__global__ void k_axpy_nodes(long long n, double c, const double* __restrict__ s,
                             double* __restrict__ psi) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    psi[e] += c * s[e];
}

// Dense nk x nk solve by Gaussian elimination with partial pivoting (nk <= 64).
static bool dense_solve(int n, std::vector<double>& A, std::vector<double>& b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[r * n + k]) > std::fabs(A[piv * n + k])) piv = r;
    if (!(std::fabs(A[piv * n + k]) > 0.0)) return false;
    if (piv != k) {
      for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[piv * n + c]);
      std::swap(b[k], b[piv]);
    }
    for (int r = k + 1; r < n; ++r) {
      const double f = A[r * n + k] / A[k * n + k];
      for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
      b[r] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double v = b[k];
    for (int c = k + 1; c < n; ++c) v -= A[k * n + c] * b[c];
    b[k] = v / A[k * n + k];
  }
  return true;
}

}  // namespace mfp

namespace mfp {

// Schedule of a Kutta sub-solve: as any solve, or with per-cell element entries.
static int kutta_schedule(const mfp_grid* grid, const mfp_solver_opts* opts, bool cells,
                          Schedule* sc) {
  if (cells) return cells_schedule(grid, opts, sc);
  return resolve_schedule(grid, opts ? opts->precision : MFP_FP64, opts, sc);
}

static size_t kutta_workspace(const mfp_grid* grid, int32_t nbody, int32_t nkutta,
                              const mfp_solver_opts* opts, bool cells) {
  if (!grid || grid->nx < 2 || grid->ny < 2 || nbody < 0 || nbody > MFP_MAX_BODIES ||
      nkutta < 0 || nkutta > nbody)
    return 0;
  Schedule sc;
  if (kutta_schedule(grid, opts, cells, &sc) != MFP_OK) return 0;
  const size_t solve = solve_layout(grid, nbody, opts ? opts->precision : MFP_FP64, nullptr,
                                    nullptr, &sc);
  const size_t nn = (size_t)(grid->nx + 1) * (grid->ny + 1);
  return ((solve + 255) & ~size_t(255)) + (size_t)nkutta * nn * sizeof(double) + 256;
}

static int kutta_drive(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                       const double* disp, const int8_t* body, const mfp_flow* flow,
                       const mfp_solver_opts* opts, const double* kutta_xy_h, int32_t pair_lo,
                       int32_t pair_hi, double* psi, double* psi_b_h, double* Q_h,
                       double* copfi_h, int64_t* kutta_node_h, mfp_stats* stats_h, void* ws,
                       size_t ws_bytes, hipStream_t st, const double* cellcoef) {
  if (!psi || !kutta_xy_h || (nbody > 0 && !psi_b_h) || pair_lo >= nbody || pair_hi >= nbody) {
    set_error("NULL argument or pair index out of range");
    return MFP_E_ARG;
  }
  if (opts->psi0) {
    set_error("no warm start with Kutta constraints");
    return MFP_E_ARG;
  }
  const mfp_grid& g = *grid;
  const double hx = grid_hx(g), hy = grid_hy(g);
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  // Kutta bodies and their nodes: the grid node nearest to the point
  std::vector<int> kb;
  std::vector<long long> kn;
  for (int b = 0; b < nbody; ++b) {
    const double px = kutta_xy_h[2 * b], py = kutta_xy_h[2 * b + 1];
    if (kutta_node_h) kutta_node_h[b] = -1;
    if (std::isnan(px) && std::isnan(py)) continue;
    if (!std::isfinite(px) || !std::isfinite(py)) {
      set_error("Kutta point of body %d is not finite", b);
      return MFP_E_ARG;
    }
    const double fi = std::floor((px - g.x0) / hx + 0.5), fj = std::floor((py - g.y0) / hy + 0.5);
    const bool side = (fi == 0 && flow->side_bc[0] != MFP_BC_NATURAL) ||
                      (fi == g.nx && flow->side_bc[1] != MFP_BC_NATURAL) ||
                      (fj == 0 && flow->side_bc[2] != MFP_BC_NATURAL) ||
                      (fj == g.ny && flow->side_bc[3] != MFP_BC_NATURAL);
    if (!(fi >= 0 && fi <= g.nx && fj >= 0 && fj <= g.ny) || side) {
      set_error("Kutta point of body %d: its node is outside the grid or on a Dirichlet side", b);
      return MFP_E_ARG;
    }
    const long long n = (long long)fj * (g.nx + 1) + (long long)fi;
    int8_t bn = 0;
    MFP_TRY_HIP(hipMemcpyAsync(&bn, body + n, 1, hipMemcpyDeviceToHost, st));
    MFP_TRY_HIP(hipStreamSynchronize(st));
    if (bn >= 0) {
      set_error("Kutta point of body %d: its node lies inside a body", b);
      return MFP_E_ARG;
    }
    kb.push_back(b);
    kn.push_back(n);
    if (kutta_node_h) kutta_node_h[b] = n;
  }
  const int nk = (int)kb.size();
  const size_t need = kutta_workspace(grid, nbody, nk, opts, cellcoef != nullptr);
  if (need == 0) {
    set_error("invalid schedule options");
    return MFP_E_ARG;
  }
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  Schedule sc;
  MFP_TRY(kutta_schedule(grid, opts, cellcoef != nullptr, &sc));
  const size_t solve_bytes = solve_layout(grid, nbody, opts->precision, nullptr, nullptr, &sc);
  double* fields = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                             ((solve_bytes + 255) & ~size_t(255)));
  unsigned long long mask = 0;
  for (int b : kb) mask |= 1ull << b;
  mfp_flow zero_flow = *flow;
  zero_flow.U = 0.0;
  // sub-solve s = 0 (S0) into psi, s = 1 + k (S_k) into fields[k]
  std::vector<double> at(((size_t)nk + 1) * (nk > 0 ? nk : 1));   // S_s(K_j)
  std::vector<double> pb(((size_t)nk + 1) * (nbody > 0 ? nbody : 1));  // S_s body values
  SolveInfo total;
  double relres_max = 0.0;
  DevState hsd0{};
  SolveWs w0;
  for (int s = 0; s <= nk; ++s) {
    SolveWs w;
    solve_layout(grid, nbody, opts->precision, ws, &w, &sc);
    w.cellcoef = cellcoef;
    w.fixed_mask = mask;
    for (int q = 0; q < nk; ++q) w.fixed[kb[q]] = (s >= 1 && q == s - 1) ? 1.0 : 0.0;
    mfp_solver_opts o = *opts;
    if (s > 0) o.estimate_kappa = 0;
    SolveInfo info;
    MFP_TRY(solve_core(g, circles_h, nbody, disp, body, s == 0 ? flow : &zero_flow, &o, nullptr,
                       false, w, st, &info));
    double* out = s == 0 ? psi : fields + (size_t)(s - 1) * nn;
    k_output<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, w.x, w.g, w.st, out,
                                                 -1, -1, 0.0, 0.0, 0.0);
    MFP_TRY_HIP(hipGetLastError());
    DevState hsd;
    MFP_TRY_HIP(hipMemcpyAsync(&hsd, w.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
    for (int j = 0; j < nk; ++j)
      MFP_TRY_HIP(hipMemcpyAsync(&at[(size_t)s * nk + j], out + kn[j], sizeof(double),
                                 hipMemcpyDeviceToHost, st));
    MFP_TRY_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < nbody; ++b) pb[(size_t)s * nbody + b] = hsd.xb[hsd.iters & 1][b];
    for (int q = 0; q < nk; ++q) pb[(size_t)s * nbody + kb[q]] = (s >= 1 && q == s - 1) ? 1.0 : 0.0;
    if (s == 0) {
      total = info;
      hsd0 = hsd;
      w0 = w;
    } else {
      total.iters += info.iters;
      total.inner += info.inner;
      total.outer += info.outer;
      total.applies += info.applies;
      total.solve_ms += info.solve_ms;
      if (info.done != 1 && total.done == 1) total.done = info.done;
      total.stagnated = total.stagnated || info.stagnated;
    }
    if (stats_h) {
      mfp_stats one;
      MFP_TRY(fill_stats(w, info, nbody, hsd, st, &one));
      relres_max = std::max(relres_max, one.relres_true);
    }
    if (info.done == 2) return finish_status(info);  // breakdown: no result
  }
  // the Kutta rows: (I - M) c = S0(K), M_jk = S_k(K_j)
  std::vector<double> c(nk);
  if (nk > 0) {
    std::vector<double> A((size_t)nk * nk), rhs(nk);
    for (int j = 0; j < nk; ++j) {
      rhs[j] = at[j];
      for (int k = 0; k < nk; ++k)
        A[(size_t)j * nk + k] = (j == k ? 1.0 : 0.0) - at[(size_t)(k + 1) * nk + j];
    }
    if (!dense_solve(nk, A, rhs)) {
      set_error("Kutta system singular");
      return MFP_E_BREAKDOWN;
    }
    c = rhs;
    for (int k = 0; k < nk; ++k) {
      k_axpy_nodes<<<grid_blocks(nn), BLOCK, 0, st>>>(nn, c[k], fields + (size_t)k * nn, psi);
      MFP_TRY_HIP(hipGetLastError());
    }
  }
  for (int b = 0; b < nbody; ++b) {
    double v = pb[b];
    for (int k = 0; k < nk; ++k) v += c[k] * pb[(size_t)(k + 1) * nbody + b];
    psi_b_h[b] = v;
  }
  if (pair_lo >= 0 && pair_hi >= 0) {
    const double Q = psi_b_h[pair_hi] - psi_b_h[pair_lo];
    if (Q_h) *Q_h = Q;
    if (copfi_h) *copfi_h = Q / (flow->U * (circles_h[pair_hi].cy - circles_h[pair_lo].cy));
  }
  MFP_TRY_HIP(hipStreamSynchronize(st));
  if (stats_h) {
    MFP_TRY(fill_stats(w0, total, nbody, hsd0, st, stats_h));
    stats_h->iters = total.iters;
    stats_h->applies = total.applies;
    stats_h->solve_ms = total.solve_ms;
    stats_h->relres_true = relres_max;
  }
  return finish_status(total);
}

}  // namespace mfp

extern "C" size_t mfp_kutta_workspace_size(const mfp_grid* grid, int32_t nbody, int32_t nkutta,
                                           const mfp_solver_opts* opts) {
  return kutta_workspace(grid, nbody, nkutta, opts, false);
}

extern "C" int mfp_psi_solve_kutta(const mfp_grid* grid, const mfp_circle* circles_h,
                                   int32_t nbody, const double* disp, const int8_t* kind,
                                   const int8_t* body, const mfp_flow* flow,
                                   const mfp_solver_opts* opts, const double* kutta_xy_h,
                                   int32_t pair_lo, int32_t pair_hi, double* psi,
                                   double* psi_b_h, double* Q_h, double* copfi_h,
                                   int64_t* kutta_node_h, mfp_stats* stats_h, void* ws,
                                   size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_solve_args(grid, circles_h, nbody, disp, kind, body, flow, opts, ws));
  return kutta_drive(grid, circles_h, nbody, disp, body, flow, opts, kutta_xy_h, pair_lo,
                     pair_hi, psi, psi_b_h, Q_h, copfi_h, kutta_node_h, stats_h, ws, ws_bytes,
                     static_cast<hipStream_t>(stream_), nullptr);
}

namespace mfp {

size_t psi_solve_cells_kutta_workspace(const mfp_grid* grid, int nbody, int nkutta,
                                       const mfp_solver_opts* opts) {
  return kutta_workspace(grid, nbody, nkutta, opts, true);
}

int psi_solve_cells_kutta(const mfp_grid* grid, const mfp_circle* circles_h, int nbody,
                          const double* disp, const int8_t* body, const double* cellcoef,
                          const mfp_flow* flow, const mfp_solver_opts* opts,
                          const double* kutta_xy_h, int pair_lo, int pair_hi, double* psi,
                          double* psi_b_h, double* Q_h, double* copfi_h, int64_t* kutta_node_h,
                          mfp_stats* stats_h, void* ws, size_t ws_bytes, hipStream_t st) {
  MFP_TRY(check_solve_args(grid, circles_h, nbody, disp, body, body, flow, opts, ws));
  if (!cellcoef) {
    set_error("NULL element entries");
    return MFP_E_ARG;
  }
  return kutta_drive(grid, circles_h, nbody, disp, body, flow, opts, kutta_xy_h, pair_lo,
                     pair_hi, psi, psi_b_h, Q_h, copfi_h, kutta_node_h, stats_h, ws, ws_bytes, st,
                     cellcoef);
}

}  // namespace mfp

extern "C" int mfp_phi_solve(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                             const double* disp, const int8_t* kind, const int8_t* body,
                             const mfp_flow* flow, const mfp_solver_opts* opts, double* phi,
                             mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_solve_args(grid, circles_h, nbody, disp, kind, body, flow, opts, ws));
  if (!phi) {
    set_error("phi is NULL");
    return MFP_E_ARG;
  }
  Schedule sc;
  MFP_TRY(resolve_schedule(grid, opts->precision, opts, &sc));
  const size_t need = solve_layout(grid, nbody, opts->precision, nullptr, nullptr, &sc);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveWs w;
  solve_layout(grid, nbody, opts->precision, ws, &w, &sc);
  w.phi = 1;
  const mfp_grid& g = *grid;
  // no body constraint (nb = 0); circle 0 only gives MFP_BC_DIRICHLET_CYLPHI its data
  SolveInfo info;
  MFP_TRY(solve_core(g, nullptr, 0, disp, body, flow, opts, nullptr, false, w, st, &info,
                     nbody > 0 ? circles_h : nullptr));
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  k_output_phi<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, body, w.x, w.g, phi);
  MFP_TRY_HIP(hipGetLastError());
  DevState hsd;
  MFP_TRY_HIP(hipMemcpyAsync(&hsd, w.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  MFP_TRY(fill_stats(w, info, 0, hsd, st, stats_h));
  return finish_status(info);
}

static size_t grad_workspace(const mfp_grid* grid, int32_t nbody, const mfp_solver_opts* o) {
  if (!grid || grid->nx < 2 || grid->ny < 2 || nbody < 0 || nbody > MFP_MAX_BODIES) return 0;
  Schedule sc;
  if (resolve_schedule(grid, o->precision, o, &sc) != MFP_OK) return 0;
  Bump bp(nullptr);
  bp.off = solve_layout(grid, nbody, o->precision, nullptr, nullptr, &sc);
  const size_t nn = (size_t)(grid->nx + 1) * (grid->ny + 1);
  bp.take<double>(nn);                                  // lambda (nodal)
  bp.take<double>(8 * (size_t)grid->nx * grid->ny);     // per-cell shape derivatives
  return bp.off + 256;
}

extern "C" size_t mfp_grad_workspace_size(const mfp_grid* grid, int32_t nbody,
                                          int32_t precision) {
  mfp_solver_opts o{};
  o.precision = precision;
  return grad_workspace(grid, nbody, &o);
}

extern "C" int mfp_psi_grad(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                            const double* disp, const int8_t* kind, const int8_t* body,
                            const mfp_flow* flow, const mfp_solver_opts* opts, const double* psi,
                            const double* psi_b_h, const double* dL_dpsib_h, double dL_dcopfi,
                            int32_t pair_lo, int32_t pair_hi, double* dL_ddisp,
                            double* dL_dcentre_h, double* dL_dU_h, mfp_stats* stats_h, void* ws,
                            size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_solve_args(grid, circles_h, nbody, disp, kind, body, flow, opts, ws));
  if (!psi || !dL_ddisp || (nbody > 0 && (!psi_b_h || !dL_dcentre_h))) {
    set_error("NULL argument");
    return MFP_E_ARG;
  }
  const bool use_pair = pair_lo >= 0 && pair_hi >= 0 && dL_dcopfi != 0.0;
  if (pair_lo >= nbody || pair_hi >= nbody || (use_pair && pair_lo == pair_hi)) {
    set_error("bad pair");
    return MFP_E_ARG;
  }
  if (!std::isfinite(dL_dcopfi)) {
    set_error("dL_dcopfi is not finite");
    return MFP_E_ARG;
  }
  Schedule sc;
  MFP_TRY(resolve_schedule(grid, opts->precision, opts, &sc));
  const size_t need = grad_workspace(grid, nbody, opts);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveWs w;
  Bump bp(ws);
  bp.off = solve_layout(grid, nbody, opts->precision, ws, &w, &sc);
  const mfp_grid& g = *grid;
  const int nb = nbody;
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  double* lam = bp.take<double>(nn);
  double* cg = bp.take<double>(8 * (size_t)g.nx * g.ny);
  // adjoint right-hand side dJ/dpsi_b and the explicit dependence of CoPFI on the
  // pair's centre heights
  double rhs[MFP_MAX_BODIES] = {0};
  for (int b = 0; b < nb; ++b) {
    rhs[b] = dL_dpsib_h ? dL_dpsib_h[b] : 0.0;
    dL_dcentre_h[2 * b] = 0.0;
    dL_dcentre_h[2 * b + 1] = 0.0;
  }
  if (use_pair) {
    const double dy = circles_h[pair_hi].cy - circles_h[pair_lo].cy;
    const double den = flow->U * dy;
    const double J = (psi_b_h[pair_hi] - psi_b_h[pair_lo]) / den;
    rhs[pair_hi] += dL_dcopfi / den;
    rhs[pair_lo] -= dL_dcopfi / den;
    dL_dcentre_h[2 * pair_hi + 1] += -dL_dcopfi * J / dy;
    dL_dcentre_h[2 * pair_lo + 1] += dL_dcopfi * J / dy;
  }
  // free stream: y = U y1, so with A lambda = dL/dy, lambda^T db/dU = (dL/dy)^T y / U;
  // the explicit U in CoPFI's denominator cancels the pair's part of it
  if (dL_dU_h) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += rhs[b] * psi_b_h[b];
    if (use_pair)
      s -= dL_dcopfi * (psi_b_h[pair_hi] - psi_b_h[pair_lo]) /
           (flow->U * (circles_h[pair_hi].cy - circles_h[pair_lo].cy));
    *dL_dU_h = flow->U != 0.0 ? s / flow->U : 0.0;
  }
  // the adjoint starts from zero whatever the caller's options say
  mfp_solver_opts ao = *opts;
  ao.psi0 = nullptr;
  SolveInfo info;
  MFP_TRY(solve_core(g, circles_h, nb, disp, body, flow, &ao, rhs, true, w, st, &info));
  // lambda as a nodal vector (Dirichlet nodes 0, body nodes lambda_b)
  k_output<<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, g.nx, g.ny, w.tag, w.x, w.g, w.st, lam, -1,
                                               -1, 1.0, 0.0, 1.0);
  const long long nc = (long long)g.nx * g.ny;
  k_shape_grad_cells<<<grid_blocks(nc), BLOCK, 0, st>>>(g.nx, g.ny, grid_hx(g), grid_hy(g), body,
                                                         disp, lam, psi, cg);
  k_shape_grad_gather<<<grid_blocks(nn), BLOCK, 0, st>>>(g.nx, g.ny, cg, dL_ddisp);
  MFP_TRY_HIP(hipGetLastError());
  DevState hsd;
  MFP_TRY_HIP(hipMemcpyAsync(&hsd, w.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  MFP_TRY(fill_stats(w, info, nb, hsd, st, stats_h));
  return finish_status(info);
}

// ---------------------------------------------------------------------------------
// Element apply without allocation (mfp_element_apply_noalloc)
// ---------------------------------------------------------------------------------
namespace mfp {

// The entry point's scratch: a file-scope device array, one copy per GPU, kept until
// the process ends.  Host code never passes its name to a kernel (in host code it is
// a stand-in, not a device address): the address comes from hipGetSymbolAddress, once
// per device, with that device current.
constexpr size_t NOALLOC_BYTES = (size_t)MFP_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Address of the current device's scratch (resolved on the first call on a device).
static int scratch_address(void** out) {
  int dev = 0;
  MFP_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    set_error("device %d beyond the %d devices the scratch table covers", dev,
              NOALLOC_MAX_DEVICES);
    return MFP_E_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return MFP_E_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MFP_OK;
}

template <typename T>
__global__ void k_zero(long long n, T* __restrict__ v) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    v[e] = (T)0;
}

// What the element apply needs and nothing else: tags, displacements / hx (FP64,
// and FP32 copies for an FP32 apply), the padded input and output, the task metadata
// and the work list (no body unknowns: the product is the full nodal K p).
static size_t noalloc_layout(const mfp_grid* g, int precision, void* base, SolveWs* out) {
  Bump bp(base);
  SolveWs w{};
  w.L = make_layout(g->nx, g->ny);
  const size_t n = (size_t)w.L.n;
  const int nt = w.L.ntasks();
  const size_t esz = precision == MFP_FP64 ? sizeof(double) : sizeof(float);
  w.tag = bp.take<int8_t>(n);
  w.dx = bp.take<double>(n);
  w.dy = bp.take<double>(n);
  if (precision != MFP_FP64) {
    w.dxf = bp.take<float>(n);
    w.dyf = bp.take<float>(n);
  }
  char* src = bp.take<char>(n * esz);
  char* dst = bp.take<char>(n * esz);
  w.tplain = bp.take<uint8_t>(nt);
  w.tbody = bp.take<unsigned long long>(nt);
  w.tslot = bp.take<int>(nt);
  w.nslots = bp.take<int>(1);
  w.segtab = bp.take<int4>((size_t)nt + 4096);
  w.part = bp.take<double>(GMAX);
  w.bstride = 64;
  w.bpart = bp.take<double>(2 * w.bstride);
  if (precision == MFP_FP64) {
    w.p0 = reinterpret_cast<double*>(src);
    w.q = reinterpret_cast<double*>(dst);
  } else {
    w.p0f = reinterpret_cast<float*>(src);
    w.qf = reinterpret_cast<float*>(dst);
  }
  if (out) {
    if (base) w.sp = seg_plan(w.L, single_target(w.L, precision));
    *out = w;
  }
  return bp.off + 256;
}

}  // namespace mfp

extern "C" int mfp_element_apply_noalloc(const mfp_grid* grid, const double* disp,
                                         const int8_t* body, int32_t precision, const void* p,
                                         void* q, void* stream_) {
  clear_error();
  MFP_TRY(check_grid(grid));
  if (!disp || !body || !p || !q) {
    set_error("NULL pointer");
    return MFP_E_ARG;
  }
  if (precision != MFP_FP64 && precision != MFP_FP32) {
    set_error("precision must be MFP_FP64 or MFP_FP32");
    return MFP_E_ARG;
  }
  const size_t need = noalloc_layout(grid, precision, nullptr, nullptr);
  if (need > NOALLOC_BYTES) {
    set_error("grid %dx%d needs %zu bytes of scratch, above the %zu of the allocation-free "
              "entry point: use mfp_element_apply with a workspace", grid->nx, grid->ny, need,
              NOALLOC_BYTES);
    return MFP_E_WORKSPACE;
  }
  const mfp_grid& g = *grid;
  {
    const Layout L = make_layout(g.nx, g.ny);
    if (L.nstrip > SEG_MAX_STRIPS || L.nchunk > 0xffff) {
      set_error("grid too large");
      return MFP_E_ARG;
    }
  }
  void* base = nullptr;
  MFP_TRY(scratch_address(&base));
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveWs w;
  noalloc_layout(grid, precision, base, &w);
  // tags and scaled displacements (k_setup writes every padded entry), task metadata
  // and the work list
  SetupArgs s{};
  s.L = w.L;
  s.nx = g.nx;
  s.ny = g.ny;
  s.x0 = g.x0;
  s.y0 = g.y0;
  s.hx = grid_hx(g);
  s.hy = grid_hy(g);
  s.inv_hx = 1.0 / s.hx;
  for (int k = 0; k < 4; ++k) s.bc[k] = MFP_BC_NATURAL;
  s.disp = disp;
  s.body = body;
  s.tag = w.tag;
  s.dx = w.dx;
  s.dy = w.dy;
  s.dxf = w.dxf;
  s.dyf = w.dyf;
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  // the padded input is zero off the nodes (halo rows and padding columns): cleared by a
  // kernel on every call (the array keeps the last call's contents)
  if (precision == MFP_FP64) {
    k_zero<double><<<grid_blocks(w.L.n), BLOCK, 0, st>>>(w.L.n, w.p0);
    k_to_padded<double><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, (const double*)p, w.p0);
  } else {
    k_zero<float><<<grid_blocks(w.L.n), BLOCK, 0, st>>>(w.L.n, w.p0f);
    k_to_padded<float><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, (const float*)p, w.p0f);
  }
  k_setup<<<grid_blocks(w.L.n), BLOCK, 0, st>>>(s);
  k_task_meta<<<(w.L.ntasks() + WAVES - 1) / WAVES, BLOCK, 0, st>>>(w.L, w.tag, w.dx, w.dy,
                                                                     w.tplain, w.tbody);
  k_assign_slots<<<1, BLOCK, 0, st>>>(w.L.ntasks(), w.tbody, w.tslot, w.nslots);
  k_seg_plan<<<1, 1024, 0, st>>>(w.L, w.tplain, w.sp.target, WAVES * w.sp.G, w.sp.tabsize,
                                 w.segtab);
  MFP_TRY_HIP(hipGetLastError());
  if (precision == MFP_FP64) {
    ApplyArgs<double> a = make_apply_args<double>(w, g, 0, w.dx, w.dy);
    a.src = w.p0;
    a.q = w.q;
    a.write_all = 1;
    launch_apply<double>(w.L.hc, w.sp.G, st, a);
    k_from_padded<double><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, w.q, (double*)q);
  } else {
    ApplyArgs<float> a = make_apply_args<float>(w, g, 0, w.dxf, w.dyf);
    a.src = w.p0f;
    a.q = w.qf;
    a.write_all = 1;
    launch_apply<float>(w.L.hc, w.sp.G, st, a);
    k_from_padded<float><<<grid_blocks(nn), BLOCK, 0, st>>>(w.L, w.qf, (float*)q);
  }
  MFP_TRY_HIP(hipGetLastError());
  return MFP_OK;
}

#include "batch.h"
