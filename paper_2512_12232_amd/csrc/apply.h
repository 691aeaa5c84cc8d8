// Matrix-free Q1 element operator on the padded node layout.
//
// Algorithm 1 (appendix) forms K p cell by cell: each cell's 4x4 matrix
// K_e = int (grad N)^T (grad N) dOmega (section "Weak formulation") acts on the cell's
// four nodal values, and the four results are summed into the nodes they belong to.
// Here the element matrix is never
// stored: each wavefront owns strips of 62 node columns (plus one halo column on
// each side) and marches up them a few node rows at a time, evaluating K_e(X_e) p_e
// for every cell touching its rows with the 2x2 Gauss rule from the node
// displacements; the neighbour values a cell needs come from the adjacent lane
// (DPP lane shifts) and from the rows already in registers.  Each output is written
// exactly once, so no atomics and no colouring of the global scatter are needed.
// Tasks whose footprint holds only free, undisplaced nodes take the assembled
// constant 9-point stencil of the rectangular cell instead (same operator, a few ulp
// apart).
#pragma once

#include <hip/hip_ext.h>

#include "mfp_internal.h"
#include "reduce.h"

namespace mfp {

template <typename T>
__device__ __forceinline__ T fast_rcp(T x);

template <>
__device__ __forceinline__ double fast_rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  return r;
}

template <>
__device__ __forceinline__ float fast_rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// y = K_e p_e for one bilinear quadrilateral.  Node order (i,j), (i+1,j), (i+1,j+1),
// (i,j+1); coordinates in units of hx: the undisplaced cell is [0,1] x [0,ry] and
// d* are the node displacements divided by hx (K_e is invariant under scaling in 2-D).
// x(xi,eta) is bilinear, so x_xi = ax + cx eta, x_eta = bx + cx xi and likewise for y;
// at each Gauss point the element integrand is grad_xi(N)^T G grad_xi(p) with
// G = adj(J) adj(J)^T / det J.
template <typename T>
__device__ __forceinline__ void cell_apply(T ry, T dx0, T dx1, T dx2, T dx3, T dy0, T dy1,
                                           T dy2, T dy3, T p0, T p1, T p2, T p3, T& y0,
                                           T& y1, T& y2, T& y3) {
  const T qt = (T)0.25;
  const T ax = qt * (((T)2 + (dx1 - dx0)) + (dx2 - dx3));
  const T bx = qt * ((dx3 - dx0) + (dx2 - dx1));
  const T cx = qt * ((dx0 - dx1) + (dx2 - dx3));
  const T ay = qt * ((dy1 - dy0) + (dy2 - dy3));
  const T by = qt * (((T)2 * ry + (dy3 - dy0)) + (dy2 - dy1));
  const T cy = qt * ((dy0 - dy1) + (dy2 - dy3));
  const T pa = qt * ((p1 - p0) + (p2 - p3));
  const T pb = qt * ((p3 - p0) + (p2 - p1));
  const T pc = qt * ((p0 - p1) + (p2 - p3));
  const T s = (T)0.57735026918962576451;
  const T cxs = cx * s, cys = cy * s, pcs = pc * s;
  // Jacobian entries: J11, J12 depend on eta only; J21, J22 on xi only.
  const T j11m = ax - cxs, j11p = ax + cxs, j12m = ay - cys, j12p = ay + cys;
  const T j21m = bx - cxs, j21p = bx + cxs, j22m = by - cys, j22p = by + cys;
  // Gauss points g = 0..3: (xi, eta) = (-,-), (+,-), (+,+), (-,+)
  const T d0 = j11m * j22m - j12m * j21m;
  const T d1 = j11m * j22p - j12m * j21p;
  const T d2 = j11p * j22p - j12p * j21p;
  const T d3 = j11p * j22m - j12p * j21m;
  // four reciprocals from one (product trick)
  const T d01 = d0 * d1, d23 = d2 * d3;
  const T inv = fast_rcp<T>(d01 * d23);
  const T i01 = inv * d23, i23 = inv * d01;
  const T r0 = i01 * d1, r1 = i01 * d0, r2 = i23 * d3, r3 = i23 * d2;
  // adj(J) adj(J)^T entries: A = J21^2 + J22^2 (xi only), C = J11^2 + J12^2 (eta only),
  // B = J11 J21 + J12 J22
  const T Am = j21m * j21m + j22m * j22m, Ap = j21p * j21p + j22p * j22p;
  const T Cm = j11m * j11m + j12m * j12m, Cp = j11p * j11p + j12p * j12p;
  const T B0 = j11m * j21m + j12m * j22m, B1 = j11m * j21p + j12m * j22p;
  const T B2 = j11p * j21p + j12p * j22p, B3 = j11p * j21m + j12p * j22m;
  // reference gradient of p: p_xi = pa + pc eta, p_eta = pb + pc xi
  const T pxm = pa - pcs, pxp = pa + pcs, pem = pb - pcs, pep = pb + pcs;
  const T qx0 = r0 * (Am * pxm - B0 * pem), qe0 = r0 * (Cm * pem - B0 * pxm);
  const T qx1 = r1 * (Ap * pxm - B1 * pep), qe1 = r1 * (Cm * pep - B1 * pxm);
  const T qx2 = r2 * (Ap * pxp - B2 * pep), qe2 = r2 * (Cp * pep - B2 * pxp);
  const T qx3 = r3 * (Am * pxp - B3 * pem), qe3 = r3 * (Cp * pem - B3 * pxp);
  // y_a = 1/4 sum_g [xi_a (1 + eta_a eta_g) qx_g + eta_a (1 + xi_a xi_g) qe_g]
  const T Sx = (qx0 + qx1) + (qx2 + qx3);
  const T Sxe = s * ((qx2 + qx3) - (qx0 + qx1));
  const T Se = (qe0 + qe1) + (qe2 + qe3);
  const T Sex = s * ((qe1 + qe2) - (qe0 + qe3));
  y0 = qt * ((Sxe - Sx) + (Sex - Se));
  y1 = qt * ((Sx - Sxe) - (Se + Sex));
  y2 = qt * ((Sx + Sxe) + (Se + Sex));
  y3 = qt * ((Se - Sex) - (Sx + Sxe));
}

// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1).  shr: lane i receives
// lane i-1 (lane 0 receives 0); shl: lane i receives lane i+1 (lane 63 receives 0).
// All 64 lanes must be active.
__device__ __forceinline__ int dpp_shr1_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shl1_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ double lane_shr(double v) {
  const int lo = dpp_shr1_i(__double2loint(v)), hi = dpp_shr1_i(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_shl(double v) {
  const int lo = dpp_shl1_i(__double2loint(v)), hi = dpp_shl1_i(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_shr(float v) {
  return __int_as_float(dpp_shr1_i(__float_as_int(v)));
}
__device__ __forceinline__ float lane_shl(float v) {
  return __int_as_float(dpp_shl1_i(__float_as_int(v)));
}
__device__ __forceinline__ int lane_shl(int v) { return dpp_shl1_i(v); }

// ---- per-task building blocks --------------------------------------------------
// A task is a 64-column strip x HC node rows; "rows" 0..HC+1 below are the task's
// HC owned rows plus one halo row on each side, held one value per lane.

// K v at rows 1..HC (qr[r-1]) of a task whose footprint is all free and undisplaced:
// the assembled 9-point stencil, horizontal neighbours by lane shifts.
// FP32 evaluates it in difference form, sum over neighbours of c_n (v_n - v), which
// the stencil's zero row sum (cC = -(2 cE + 2 cN + 4 cD)) makes equal to the plain
// form.  For a smooth v the plain form subtracts terms of size |c||v| that nearly
// cancel, so its relative error grows like eps / (h k)^2 for a mode of wavenumber k
// (order one for the lowest modes at 4096x2048 in FP32), whereas neighbour
// differences of nearby values are exact or nearly so: eps / (h k).  The FP32
// iteration then sees the low modes of K almost as FP64 does.  The geometric path
// (cell_apply) works on differences of p already.
template <typename T, int HC>
__device__ __forceinline__ void stencil_task(T cC, T cE, T cN, T cD, const T (&v)[HC + 2],
                                             T (&qr)[HC]) {
#pragma unroll
  for (int r = 1; r <= HC; ++r) {
    if constexpr (sizeof(T) == 4) {
      const T a = v[r];
      const T dv = (v[r - 1] - a) + (v[r + 1] - a);  // vertical neighbours
      const T dl = lane_shr(a) - a, dr = lane_shl(a) - a;
      // diagonal neighbours: the left (right) column's vertical differences plus
      // twice that column's own difference
      const T dd = (lane_shr(dv) + lane_shl(dv)) + (T)2 * (dl + dr);
      qr[r - 1] = cE * (dl + dr) + cN * dv + cD * dd;
    } else {
      const T csum = v[r - 1] + v[r + 1];
      const T pl = lane_shr(v[r]), pr = lane_shl(v[r]);
      const T csl = lane_shr(csum), csr = lane_shl(csum);
      qr[r - 1] = cC * v[r] + cE * (pl + pr) + cN * csum + cD * (csl + csr);
    }
  }
}

// K v at rows 1..HC of any task: march over the HC+1 cell rows touching its rows.
// Lane c evaluates cell (c, sr) from its own nodes and those of lane c+1 (shifted in),
// keeps the cell's contributions to its own column and shifts the contributions to
// column c+1 over; node row sr is complete once cell rows sr-1 and sr are done.
// Cells with a halo node, and cells whose four nodes lie in one body, are skipped.
template <typename T, int HC>
__device__ __forceinline__ void march_task(T ry, int lane, const int8_t (&tg)[HC + 2],
                                           const T (&v)[HC + 2], const T (&ddx)[HC + 2],
                                           const T (&ddy)[HC + 2], T (&qr)[HC]) {
  // lower node row of the current cell row (own column and right neighbour)
  int8_t g0 = tg[0];
  T p0 = v[0], x0 = ddx[0], y0 = ddy[0];
  int8_t g1n = (int8_t)lane_shl((int)g0);
  T p1n = lane_shl(p0), x1n = lane_shl(x0), y1n = lane_shl(y0);
  T carry = (T)0;
#pragma unroll
  for (int sr = 0; sr <= HC; ++sr) {
    const int8_t g3 = tg[sr + 1];
    const T p3 = v[sr + 1], x3 = ddx[sr + 1], y3 = ddy[sr + 1];
    const int8_t g2 = (int8_t)lane_shl((int)g3);
    const T p2 = lane_shl(p3), x2 = lane_shl(x3), y2 = lane_shl(y3);
    // cell (own column, row sr): nodes 0 = (c, sr), 1 = (c+1, sr), 2 = (c+1, sr+1),
    // 3 = (c, sr+1)
    const bool halo =
        (g0 == TAG_HALO) | (g1n == TAG_HALO) | (g2 == TAG_HALO) | (g3 == TAG_HALO);
    const bool inside = tag_body(g0) & (g1n == g0) & (g2 == g0) & (g3 == g0);
    T c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    if (!halo && !inside && lane < 63)
      cell_apply<T>(ry, x0, x1n, x2, x3, y0, y1n, y2, y3, p0, p1n, p2, p3, c0, c1, c2, c3);
    const T acc = carry + c0 + lane_shr(c1);
    carry = c3 + lane_shr(c2);
    if (sr >= 1) qr[sr - 1] = acc;
    g0 = g3;
    p0 = p3;
    x0 = x3;
    y0 = y3;
    g1n = g2;
    p1n = p2;
    x1n = x2;
    y1n = y2;
  }
}

// ---- element matrices evaluated once per solve ---------------------------------
// A cell's K_e is symmetric with zero row sums (K_e applied to a constant is zero),
// so its six off-diagonal entries determine it: (K_e p)_a = sum_{b != a} k_ab (p_b - p_a).
// For tasks that evaluate geometry, the iteration can read those six numbers per cell
// instead of rebuilding the Jacobians from the displacements every iteration: the
// same 2x2 Gauss rule (cell_apply) evaluates them once per solve, in FP64.  A task's
// slab holds cell rows 0..HC (the rows touching its node rows) x the six entries
// (k01, k02, k03, k12, k13, k23) x 64 lanes, lane-contiguous; lane c holds cell
// (c, row) between node columns c and c+1, lane 63 and cells with a halo node or
// inside a body hold zeros (they contribute nothing).
constexpr int KCOEF = 6;

template <int HC>
__host__ __device__ constexpr int kslab() { return (HC + 1) * KCOEF * 64; }

// The six off-diagonal entries of one cell's K_e: its columns are K_e applied to the
// unit vectors.
__device__ __forceinline__ void cell_coefficients(double ry, double x0, double x1, double x2,
                                                  double x3, double y0, double y1, double y2,
                                                  double y3, double (&k)[KCOEF]) {
  double c0, c1, c2, c3;
  cell_apply<double>(ry, x0, x1, x2, x3, y0, y1, y2, y3, 0.0, 1.0, 0.0, 0.0, c0, c1, c2, c3);
  k[0] = c0;  // k01
  cell_apply<double>(ry, x0, x1, x2, x3, y0, y1, y2, y3, 0.0, 0.0, 1.0, 0.0, c0, c1, c2, c3);
  k[1] = c0;  // k02
  k[3] = c1;  // k12
  cell_apply<double>(ry, x0, x1, x2, x3, y0, y1, y2, y3, 0.0, 0.0, 0.0, 1.0, c0, c1, c2, c3);
  k[2] = c0;  // k03
  k[4] = c1;  // k13
  k[5] = c2;  // k23
}

// K v at rows 1..HC from the task's stored element entries kc[cell row][entry] (the
// march of march_task with the cell product in difference form).
template <typename T, int HC>
__device__ __forceinline__ void march_task_stored(const T (&v)[HC + 2], const T (&kc)[HC + 1][KCOEF],
                                                  T (&qr)[HC]) {
  T p0 = v[0];
  T p1 = lane_shl(p0);
  T carry = (T)0;
#pragma unroll
  for (int sr = 0; sr <= HC; ++sr) {
    const T p3 = v[sr + 1];
    const T p2 = lane_shl(p3);
    const T d01 = p1 - p0, d02 = p2 - p0, d03 = p3 - p0;
    const T d12 = p2 - p1, d13 = p3 - p1, d23 = p3 - p2;
    const T k01 = kc[sr][0], k02 = kc[sr][1], k03 = kc[sr][2];
    const T k12 = kc[sr][3], k13 = kc[sr][4], k23 = kc[sr][5];
    const T c0 = (k01 * d01 + k02 * d02) + k03 * d03;
    const T c1 = (k12 * d12 + k13 * d13) - k01 * d01;
    const T c2 = k23 * d23 - (k02 * d02 + k12 * d12);
    const T c3 = -((k03 * d03 + k13 * d13) + k23 * d23);
    const T acc = carry + c0 + lane_shr(c1);
    carry = c3 + lane_shr(c2);
    if (sr >= 1) qr[sr - 1] = acc;
    p0 = p3;
    p1 = p2;
  }
}

// Element entries of every geometry task (tgeo[t] = its slab, -1 for constant-stencil
// tasks): one wavefront per task, geometry from the FP64 displacements / hx.
template <typename T, int HC>
__global__ void __launch_bounds__(256) k_elem_coef(Layout L, double ry,
                                                   const int8_t* __restrict__ tag,
                                                   const double* __restrict__ dx,
                                                   const double* __restrict__ dy,
                                                   const int* __restrict__ tgeo,
                                                   T* __restrict__ kcoef) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= L.ntasks()) return;
  const int s = tgeo[t];
  if (s < 0) return;  // uniform over the wavefront
  const int m = t % L.nstrip, kc = t / L.nstrip;
  const long long base =
      (long long)(kc * HC) * L.P + (long long)m * 64 + lane + halo_shift(lane, m, L.nstrip);
  int8_t g0 = tag[base];
  double x0 = dx[base], y0 = dy[base];
  int8_t g1 = (int8_t)lane_shl((int)g0);
  double x1 = lane_shl(x0), y1 = lane_shl(y0);
  T* out = kcoef + (size_t)s * kslab<HC>();
  for (int sr = 0; sr <= HC; ++sr) {
    const long long gi = base + (long long)(sr + 1) * L.P;
    const int8_t g3 = tag[gi];
    const double x3 = dx[gi], y3 = dy[gi];
    const int8_t g2 = (int8_t)lane_shl((int)g3);
    const double x2 = lane_shl(x3), y2 = lane_shl(y3);
    const bool halo =
        (g0 == TAG_HALO) | (g1 == TAG_HALO) | (g2 == TAG_HALO) | (g3 == TAG_HALO);
    const bool inside = tag_body(g0) & (g1 == g0) & (g2 == g0) & (g3 == g0);
    double k[KCOEF] = {0, 0, 0, 0, 0, 0};
    if (!halo && !inside && lane < 63) cell_coefficients(ry, x0, x1, x2, x3, y0, y1, y2, y3, k);
#pragma unroll
    for (int e = 0; e < KCOEF; ++e) out[(sr * KCOEF + e) * 64 + lane] = (T)k[e];
    g0 = g3;
    x0 = x3;
    y0 = y3;
    g1 = g2;
    x1 = x2;
    y1 = y2;
  }
}

// Element entries of every geometry task copied from a per-cell table of six entries
// per cell, entry-major (tab[e nx ny + j nx + i] for cell (i, j), corners counter-
// clockwise from node (i, j)): for meshes whose cells are not plain bilinear
// quadrilaterals of the displaced nodes.  Lane c's cell lies between its node column
// and the next lane's; lanes and rows without a cell of the grid get zeros.
template <typename T, int HC>
__global__ void __launch_bounds__(256) k_cells_to_slab(Layout L, const double* __restrict__ tab,
                                                       const int* __restrict__ tgeo,
                                                       T* __restrict__ kcoef) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= L.ntasks()) return;
  const int s = tgeo[t];
  if (s < 0) return;  // uniform over the wavefront
  const int m = t % L.nstrip, kc = t / L.nstrip;
  const int ci = column_node(m * 64 + lane + halo_shift(lane, m, L.nstrip));
  const bool col_ok = lane < 63 && ci >= 0 && ci < L.nx;
  const long long nc = (long long)L.nx * L.ny;
  T* out = kcoef + (size_t)s * kslab<HC>();
  for (int sr = 0; sr <= HC; ++sr) {
    const int cj = kc * HC + sr - 1;
    const bool ok = col_ok && cj >= 0 && cj < L.ny;
    const long long c = ok ? (long long)cj * L.nx + ci : 0;
#pragma unroll
    for (int e = 0; e < KCOEF; ++e)
      out[(sr * KCOEF + e) * 64 + lane] = ok ? (T)tab[e * nc + c] : (T)0;
  }
}

// Slabs for the geometry tasks, numbered in task order (single block).
__global__ void k_assign_geo(int ntiles, const uint8_t* __restrict__ tplain,
                             int* __restrict__ tgeo, int* __restrict__ ngeo) {
  __shared__ int s_scan[256];
  __shared__ int s_base;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < ntiles; c0 += 256) {
    const int t = c0 + threadIdx.x;
    const int f = (t < ntiles && !tplain[t]) ? 1 : 0;
    s_scan[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int v = threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0;
      __syncthreads();
      s_scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (t < ntiles) tgeo[t] = f ? s_base + s_scan[threadIdx.x] - 1 : -1;
    __syncthreads();
    if (threadIdx.x == 255) s_base += s_scan[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ngeo = s_base;
}

// Per-body sums of one node row: lane b of the wavefront accumulates the sum of `val`
// over the owned nodes of body b in this row (fixed order).
__device__ __forceinline__ void body_row(bool owner, int8_t g, double val, int lane,
                                         double& bacc) {
  unsigned long long rowb = __ballot(owner && g >= TAG_BODY0);
  while (rowb) {
    const int src = __ffsll((long long)rowb) - 1;
    const int bt = __shfl((int)g, src, 64);
    const bool mine = owner && g == bt;
    const double bv = wave_sum(mine ? val : 0.0);
    if (lane == bt - TAG_BODY0) bacc += bv;
    rowb &= ~__ballot(mine);
  }
}

template <typename T>
struct ApplyArgs {
  int P, nstrip;                 // pitch, strips (task t = chunk * nstrip + strip)
  const int4* segtab;            // work list: x = strip, y = first chunk | (length << 16),
                                 // (z, w) = mask of constant-stencil tasks
  int tabsize;                   // entries (a multiple of 4 G; empty entries have length 0)
  const int8_t* tag;
  const T* dx;                   // displacement / hx
  const T* dy;
  const uint8_t* tplain;         // per task, 1: constant-stencil task
  const unsigned long long* tbody;  // per task: bodies among its owned nodes
  const int* tslot;              // per task: body-partial slot or -1
  const T* src;                  // p (zero at halo nodes)
  T* q;                          // K p at free nodes (all in-domain nodes if write_all)
  double* part;                  // per-block partial of p.q over free nodes
  double* bpart;                 // per-slot, per-body partial sums of K p
  int nb;
  int write_all;
  T cC, cE, cN, cD;              // constant stencil (centre, east/west, north/south, diag)
  T ry;                          // hy / hx
  int G;                         // blocks of this apply (batched launches)
  const int* skip;               // return at once when *skip != 0
  const T* kcoef;                // non-null: geometry tasks read stored element entries
  const int* tgeo;               // per task: its slab of kcoef, -1 for constant-stencil tasks
};

// q = K src, with per-block partials of src.q over free nodes and per-slot body sums.
//
// Work unit: a task is a 64-column strip x HC node rows; a wavefront takes a segment
// of consecutive tasks of one strip from the work list (segments of about equal cost)
// and marches upward through them.  The
// two node rows that consecutive tasks share stay in registers, and the residual and
// direction rows of the next task are requested before the current one is computed,
// so every wavefront keeps a task's worth of loads in flight.
// Constant-stencil tasks evaluate the assembled 9-point stencil with lane shifts for
// the horizontal neighbours.  Other tasks march over the HC+1 cell rows touching their
// rows: lane c evaluates cell (c, j) from its own nodes and those of lane c+1 (shifted
// in), keeps the cell's contributions to its own column and shifts the contributions
// to column c+1 over; node (c, j) is complete once cell rows j-1 and j are done.
template <typename T, int HC>
__device__ __forceinline__ void apply_core(const ApplyArgs<T>& a, const int vblk, const int G,
                                           double* s_red) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  // consecutive virtual blocks share an XCD (work-groups are dealt round-robin to 8 XCDs;
  // vblk and blockIdx.x agree modulo 8)
  const int vb = (vblk & 7) * (G >> 3) + (vblk >> 3);
  if (a.skip && *a.skip) return;
  const T* src = a.src;
  const long long P = a.P;
  const int nstrip = a.nstrip;
  const bool owner = lane >= 1 && lane <= SW;
  const int W = G * WAVES;

  // segment state: strip, chunk range, constant-stencil mask (bit i: task kc0 + i)
  int s = vb * WAVES + wv;
  int m = 0, kc0 = 0, kc1 = 0;
  unsigned long long plain_mask = 0ull;
  int fl_body = 0, slot_l = -1;                // this lane's task (kc0 + lane)
  T f0s = 0, f1s = 0;                          // rows 0, 1 of the segment's first task
  T ns[HC];                                    // rows 2..HC+1 of the next task
  int8_t tg[HC + 2];                           // tags and displacements of the current
  T ddx[HC + 2], ddy[HC + 2];                  // task (tasks that evaluate geometry)
  int shift = 0;  // this lane's read column minus its own column (halo lanes)
  auto load_geom = [&](long long base) {
#pragma unroll
    for (int r = 0; r < HC + 2; ++r) {
      tg[r] = a.tag[base + shift + r * P];
      ddx[r] = a.dx[base + shift + r * P];
      ddy[r] = a.dy[base + shift + r * P];
    }
  };
  auto seg_load = [&](int sg) {
    const int4 e = a.segtab[sg];
    m = e.x;
    kc0 = e.y & 0xffff;
    kc1 = kc0 + (e.y >> 16);
    plain_mask = (unsigned long long)(unsigned)e.z | ((unsigned long long)(unsigned)e.w << 32);
    if (kc1 <= kc0) return;
    const int kcl = min(kc0 + lane, kc1 - 1);
    const int tl = kcl * nstrip + m;
    fl_body = a.tbody[tl] != 0ull;
    slot_l = a.tslot[tl];
    shift = halo_shift(lane, m, nstrip);
    const long long base = (long long)(kc0 * HC) * P + (long long)m * 64 + lane;
    const long long lb = base + shift;
    f0s = src[lb];
    f1s = src[lb + P];
#pragma unroll
    for (int r = 0; r < HC; ++r) {
      ns[r] = src[lb + (r + 2) * P];
    }
    // the first task's geometry travels with its rows
    if (!(plain_mask & 1ull)) load_geom(base);
  };
  bool loaded = false;
  if (s < a.tabsize) {
    seg_load(s);
    loaded = true;
  }

  double pq = 0.0;
  for (; s < a.tabsize; s += W) {
    if (!loaded) seg_load(s);  // later entries of this wavefront
    loaded = false;
    if (kc1 <= kc0) continue;
    const unsigned long long body_mask = __ballot(fl_body != 0);
    T v[HC + 2];  // input vector at rows 0..HC+1 of the task
    v[0] = f0s;
    v[1] = f1s;
    for (int kc = kc0; kc < kc1; ++kc) {
      const int it = kc - kc0;
      const bool first = kc == kc0;
      // local row r = 0 .. HC+1 is padded row kc*HC + r; lane is padded column m*64+lane
      const long long base = (long long)(kc * HC) * P + (long long)m * 64 + lane;
      const bool plain = (plain_mask >> it) & 1ull;
      // rows 2..HC+1 arrived with the previous prefetch
#pragma unroll
      for (int r = 0; r < HC; ++r) v[r + 2] = ns[r];
      // requested before the next task's rows, so that waiting for them does not wait
      // for the prefetch
      if (!plain && !first) load_geom(base);
      if (kc + 1 < kc1) {
        // rows 2..HC+1 of the next task: padded rows (kc+1)*HC + 2 ..
#pragma unroll
        for (int r = 0; r < HC; ++r) ns[r] = src[base + shift + (HC + 2 + r) * P];
      }
      T qr[HC];
      const bool bm = !plain && ((body_mask >> it) & 1ull);
      if (plain) {
        stencil_task<T, HC>(a.cC, a.cE, a.cN, a.cD, v, qr);
      } else if (a.kcoef) {
        T kcv[HC + 1][KCOEF];
        const T* kb = a.kcoef + (size_t)a.tgeo[kc * nstrip + m] * kslab<HC>() + lane;
#pragma unroll
        for (int r = 0; r <= HC; ++r)
#pragma unroll
          for (int e = 0; e < KCOEF; ++e) kcv[r][e] = kb[(r * KCOEF + e) * 64];
        march_task_stored<T, HC>(v, kcv, qr);
      } else {
        march_task<T, HC>(a.ry, lane, tg, v, ddx, ddy, qr);
      }
      double bacc = 0.0;  // lane b accumulates body b of this task
#pragma unroll
      for (int r = 1; r <= HC; ++r) {
        const long long gi = base + r * P;
        const int8_t g = plain ? (int8_t)TAG_FREE : tg[r];
        const T qv = qr[r - 1];
        const bool fr = tag_own(g);  // free (the potential's body nodes too)
        // every lane stores (the padding lanes zeros): whole aligned rows
        const bool keep = owner && (fr || (a.write_all && g != TAG_HALO));
        a.q[gi] = keep ? qv : (T)0;
        if (owner && fr) pq += (double)v[r] * (double)qv;
        if (bm) body_row(owner, g, (double)qv, lane, bacc);
      }
      if (bm) {
        const int slot = __shfl(slot_l, it, 64);  // whole wavefront active here
        if (lane < a.nb) a.bpart[(long long)slot * a.nb + lane] = bacc;
      }
      v[0] = v[HC];
      v[1] = v[HC + 1];
    }
  }
  const double bsum = block_sum(pq, s_red);
  if (tid == 0) a.part[vblk] = bsum;
}

template <typename T, int HC>
__global__ void __launch_bounds__(BLOCK) k_apply(ApplyArgs<T> a) {
  __shared__ double s_red[WAVES];
  apply_core<T, HC>(a, blockIdx.x, gridDim.x, s_red);
}

// Many independent systems in one launch: block b works for system map[b].x as its
// virtual block map[b].y (each system's blocks start at a multiple of 8).
template <typename T, int HC>
__global__ void __launch_bounds__(BLOCK) k_apply_batch(const ApplyArgs<T>* __restrict__ args,
                                                       const int2* __restrict__ map) {
  __shared__ double s_red[WAVES];
  const int2 vm = map[blockIdx.x];
  const ApplyArgs<T>& a = args[vm.x];
  apply_core<T, HC>(a, vm.y, a.G, s_red);
}

// Launch the apply for the layout's task height.  With events, they are recorded by
// the runtime at the start and end of this kernel's execution (hipExtLaunchKernel),
// so their difference is the kernel's own duration.
template <typename T>
inline void launch_apply(int hc, int G, hipStream_t st, const ApplyArgs<T>& a,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (e0) {
    if (hc == 4)
      hipExtLaunchKernelGGL(k_apply<T, 4>, dim3(G), dim3(BLOCK), 0, st, e0, e1, 0, a);
    else if (hc == 5)
      hipExtLaunchKernelGGL(k_apply<T, 5>, dim3(G), dim3(BLOCK), 0, st, e0, e1, 0, a);
    else
      hipExtLaunchKernelGGL(k_apply<T, 8>, dim3(G), dim3(BLOCK), 0, st, e0, e1, 0, a);
    return;
  }
  if (hc == 4)
    k_apply<T, 4><<<G, BLOCK, 0, st>>>(a);
  else if (hc == 5)
    k_apply<T, 5><<<G, BLOCK, 0, st>>>(a);
  else
    k_apply<T, 8><<<G, BLOCK, 0, st>>>(a);
}

// Per-body sums of the slot partials, into s_qb[0 .. nb); wave w handles bodies
// w, w+4, ...  Fixed order.  The first 64 slots of every body are requested at once
// (the partial buffer always holds at least 64 slots), so the common case costs one
// memory round trip.
__device__ __forceinline__ void body_sums(const double* __restrict__ bpart, int nslots, int nb,
                                          double* s_qb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int b = w; b < nb; b += BLOCK / 64) {
    double v = bpart[(long long)lane * nb + b];
    v = lane < nslots ? v : 0.0;
    for (int sl = lane + 64; sl < nslots; sl += 64) v += bpart[(long long)sl * nb + b];
    v = wave_sum(v);
    if (lane == 0) s_qb[b] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ void body_sums(const double* __restrict__ bpart,
                                          const int* __restrict__ nslots_p, int nb,
                                          double* s_qb) {
  body_sums(bpart, *nslots_p, nb, s_qb);
}

}  // namespace mfp
