// The paper's mixed-cell mesh on the GPU and the stream-function solve on it
// (section "Body-Conforming Grid Generation": grid points just inside a body moved
// onto it along grid lines, node splitting, triangles and pentagons, pentagons cut
// into a triangle and a quadrilateral; section "Weak formulation": element
// matrices of triangles and quadrilaterals; Algorithm 1: CG with the body values as
// constrained unknowns).
//
// Mesh (one thread per node, edge or cell; no atomics in what is written):
//   k_mx_classify   node -> body by (x-cx)^2 + (y-cy)^2 <= r^2 in FP64
//   k_mx_edge_flags an edge joining an inside and a fluid node is cut (flag 1);
//                   an edge joining two bodies is an error
//   (scan)          cut points numbered in edge order: horizontal edges, then vertical
//   k_mx_cut        the cut point I + t (O - I), |I - c + t (O - I)| = r, t in [0, 1)
//   k_mx_sweep_multi Jacobi sweeps of the displacement on fluid nodes, up to 8 per
//                   launch on LDS tiles; an inside neighbour contributes its cut point's
//                   displacement P - I.  Sweep k covers the box of the fluid nodes next
//                   to a cut edge widened by k nodes: outside it every displacement is
//                   still zero
//   k_mx_cell_count elements per cell (0, 1 or 2), errors for cells touching two bodies;
//                   a cell whose inside and fluid corners alternate (a thin part of a
//                   body crosses it) gets a triangle at each fluid corner
//   (scan)          elements numbered in cell order
//   k_mx_cells      the polygon of each cell: fluid corners and cut points walked
//                   counter-clockwise from corner (i, j); pentagons split from the cut
//                   point after the inside corner; slivers (two cut points within
//                   1e-12 h, max norm) not meshed
// Apply: element matrices (P1 triangles exactly, Q1 quadrilaterals by 2x2 Gauss)
// evaluated once per call into the workspace (the paper stores them); q = K p is a
// gather: every mixed node sums, in a fixed order, its rows of the elements of the
// (at most four) cells around it, so the result is deterministic and no scatter or
// atomic is needed.
//
// Mixed-node numbering: background nodes j (nx+1) + i (inside ones unused), then
// the cut points.  Every floating-point expression of the mesh is evaluated without
// contraction into fused multiply-adds (same rounding as a plain IEEE evaluation).
#include <cmath>
#include <cstring>
#include <vector>

#include "mfp_internal.h"
#include "reduce.h"

#pragma clang fp contract(off)

namespace mfp {
namespace mixed {

constexpr int MB = 256;  // threads per block
constexpr int SCAN_CH = MB * 8;  // flags per block of the scans
constexpr double SLIVER = 1e-12;

struct G {
  int nx, ny;
  double x0, y0, hx, hy;
  __host__ __device__ long long nn() const { return (long long)(nx + 1) * (ny + 1); }
  __host__ __device__ long long nh() const { return (long long)(ny + 1) * nx; }
  __host__ __device__ long long nv() const { return (long long)ny * (nx + 1); }
  __host__ __device__ long long nc() const { return (long long)nx * ny; }
};

__device__ __forceinline__ double node_x(const G& g, int i) { return g.x0 + (double)i * g.hx; }
__device__ __forceinline__ double node_y(const G& g, int j) { return g.y0 + (double)j * g.hy; }

static int blocks_for(long long n) {
  long long b = (n + MB - 1) / MB;
  if (b > 65535) b = 65535;
  return (int)(b < 1 ? 1 : b);
}

// ---- exclusive scan of int flags: out[k] = sum of in[0..k), out[n] = total ----------
__global__ void k_scan_block_sums(const int* __restrict__ in, long long n, int* __restrict__ bs) {
  __shared__ int s[MB];
  const long long b0 = (long long)blockIdx.x * SCAN_CH;
  int acc = 0;
  for (int k = 0; k < 8; ++k) {
    const long long i = b0 + (long long)threadIdx.x * 8 + k;
    if (i < n) acc += in[i];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = MB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bs[blockIdx.x] = s[0];
}

// single block: exclusive scan of the block sums in place, total in bs[nb]
__global__ void k_scan_sums(int* __restrict__ bs, int nb) {
  __shared__ int s[MB];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += MB) {
    const int i = c0 + threadIdx.x;
    const int v = i < nb ? bs[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < MB; off <<= 1) {
      const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bs[i] = base + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == MB - 1) base += s[MB - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) bs[nb] = base;
}

__global__ void k_scan_write(const int* __restrict__ in, long long n, const int* __restrict__ bs,
                             int nb, int* __restrict__ out) {
  __shared__ int s[MB];
  const long long b0 = (long long)blockIdx.x * SCAN_CH;
  int v[8];
  int acc = 0;
  for (int k = 0; k < 8; ++k) {
    const long long i = b0 + (long long)threadIdx.x * 8 + k;
    v[k] = i < n ? in[i] : 0;
    acc += v[k];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < MB; off <<= 1) {
    const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int run = bs[blockIdx.x] + s[threadIdx.x] - acc;
  for (int k = 0; k < 8; ++k) {
    const long long i = b0 + (long long)threadIdx.x * 8 + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = bs[nb];
}

static int scan_blocks(long long n) { return (int)((n + SCAN_CH - 1) / SCAN_CH); }

static int exclusive_scan(const int* in, long long n, int* bs, int* out, hipStream_t st) {
  const int nb = scan_blocks(n < 1 ? 1 : n);
  k_scan_block_sums<<<nb, MB, 0, st>>>(in, n, bs);
  k_scan_sums<<<1, MB, 0, st>>>(bs, nb);
  k_scan_write<<<nb, MB, 0, st>>>(in, n, bs, nb, out);
  MFP_TRY_HIP(hipGetLastError());
  return MFP_OK;
}

// ---- mesh -----------------------------------------------------------------------------
// A body on the device: a circle (x, y, r), or a Joukowski airfoil placed at (x, y)
// with map constant c (c2 = c^2), generating circle centre (xi0, eta0), R2 = R^2 and
// the rotation's cos / sin (from the host's C library).
struct MxBody {
  int kind;
  double x, y, r;
  double xi0, eta0, c2, R2, ca, sa;
};

// Airfoil level |zeta - zeta0|^2 - R^2 (<= 0 in the body) with zeta the preimage of
// (X, Y) farther from zeta0: the roots (w +- s)/2 of zeta^2 - w zeta + c^2, s a square
// root of w^2 - 4 c^2 in the stable real form (branch chosen by the sign of its real
// part).  The map is one to one from outside the circle onto outside the airfoil, so
// a point is outside iff one preimage is outside the circle.
__device__ double airfoil_level(const MxBody& b, double X, double Y) {
  const double dx = X - b.x, dy = Y - b.y;
  const double wr = b.ca * dx - b.sa * dy;
  const double wi = b.sa * dx + b.ca * dy;
  const double ar = wr * wr - wi * wi - 4.0 * b.c2;
  const double ai = 2.0 * wr * wi;
  const double m = sqrt(ar * ar + ai * ai);
  double sr, si;
  if (ar >= 0.0) {
    sr = sqrt((m + ar) * 0.5);
    si = sr > 0.0 ? ai / (2.0 * sr) : 0.0;
  } else {
    si = copysign(sqrt((m - ar) * 0.5), ai);
    sr = si != 0.0 ? ai / (2.0 * si) : 0.0;
  }
  const double e1r = (wr + sr) * 0.5 - b.xi0, e1i = (wi + si) * 0.5 - b.eta0;
  const double e2r = (wr - sr) * 0.5 - b.xi0, e2i = (wi - si) * 0.5 - b.eta0;
  const double d1 = e1r * e1r + e1i * e1i, d2 = e2r * e2r + e2i * e2i;
  return (d1 >= d2 ? d1 : d2) - b.R2;
}

__device__ __forceinline__ bool body_contains(const MxBody& b, double x, double y) {
  if (b.kind == MFP_BODY_JOUKOWSKI) return airfoil_level(b, x, y) <= 0.0;
  const double dx = x - b.x, dy = y - b.y;
  return dx * dx + dy * dy <= b.r * b.r;
}

__global__ void k_mx_classify(G g, const MxBody* __restrict__ bodies, int nb,
                              int8_t* __restrict__ body) {
  const long long nn = g.nn();
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn;
       n += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(n / (g.nx + 1)), i = (int)(n - (long long)j * (g.nx + 1));
    const double x = node_x(g, i), y = node_y(g, j);
    int b_in = -1;
    for (int b = 0; b < nb; ++b)
      if (body_contains(bodies[b], x, y)) b_in = b;
    body[n] = (int8_t)b_in;
  }
}

// Edge e: horizontal (i,j)-(i+1,j) for e < nh (e = j nx + i), vertical (i,j)-(i,j+1)
// for e = nh + j (nx+1) + i.  Ends a (lower-left) and c.
__device__ __forceinline__ void edge_ends(const G& g, long long e, int& ia, int& ja, int& ic,
                                          int& jc) {
  const long long nh = g.nh();
  if (e < nh) {
    ja = (int)(e / g.nx);
    ia = (int)(e - (long long)ja * g.nx);
    ic = ia + 1;
    jc = ja;
  } else {
    const long long v = e - nh;
    ja = (int)(v / (g.nx + 1));
    ia = (int)(v - (long long)ja * (g.nx + 1));
    ic = ia;
    jc = ja + 1;
  }
}

__global__ void k_mx_edge_flags(G g, const int8_t* __restrict__ body, int* __restrict__ flag,
                                int* __restrict__ err) {
  const long long ne = g.nh() + g.nv();
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
       e += (long long)gridDim.x * blockDim.x) {
    int ia, ja, ic, jc;
    edge_ends(g, e, ia, ja, ic, jc);
    const int ba = body[(long long)ja * (g.nx + 1) + ia];
    const int bc = body[(long long)jc * (g.nx + 1) + ic];
    if (ba >= 0 && bc >= 0 && ba != bc) err[0] = 1;  // an edge joining two bodies
    flag[e] = (ba >= 0) != (bc >= 0) ? 1 : 0;
  }
}

// t in [0, 1) with |u + t v| = r (|u| <= r < |u + v|): the oracle's expression.
__device__ __forceinline__ double edge_root(double ux, double uy, double vx, double vy, double r) {
  const double vv = vx * vx + vy * vy;
  const double uv = ux * vx + uy * vy;
  const double uu = ux * ux + uy * uy;
  return (-uv + sqrt(uv * uv - vv * (uu - r * r))) / vv;
}

// Cut point parameter t of the edge from inside node (xi, yi) along (vx, vy): for a
// circle the root of |I + t v - c| = r; for an airfoil the bracket of the first sign
// change of the level among t = k/64, bisected 60 times (the lower, inside end kept).
__device__ double cut_param(const MxBody& b, double xi, double yi, double vx, double vy) {
  if (b.kind != MFP_BODY_JOUKOWSKI) return edge_root(xi - b.x, yi - b.y, vx, vy, b.r);
  int k = 0;
  while (k < 63 && !(airfoil_level(b, xi + ((double)(k + 1) / 64.0) * vx,
                                   yi + ((double)(k + 1) / 64.0) * vy) > 0.0))
    ++k;
  double lo = (double)k / 64.0, hi = (double)(k + 1) / 64.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (airfoil_level(b, xi + mid * vx, yi + mid * vy) > 0.0)
      hi = mid;
    else
      lo = mid;
  }
  return lo;
}

__global__ void k_mx_cut(G g, const MxBody* __restrict__ circ, const int8_t* __restrict__ body,
                         const int* __restrict__ flag, const int* __restrict__ off,
                         int* __restrict__ hpt, int* __restrict__ vpt, double* __restrict__ pxy,
                         int8_t* __restrict__ pbody, int* __restrict__ pedge, long long cap) {
  const long long nh = g.nh(), ne = nh + g.nv();
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = flag[e] ? off[e] : -1;
    if (e < nh)
      hpt[e] = k;
    else
      vpt[e - nh] = k;
    if (k < 0 || k >= cap) continue;
    int ia, ja, ic, jc;
    edge_ends(g, e, ia, ja, ic, jc);
    const int ba = body[(long long)ja * (g.nx + 1) + ia];
    const bool a_in = ba >= 0;
    const int ii = a_in ? ia : ic, ji = a_in ? ja : jc;  // inside end
    const int io = a_in ? ic : ia, jo = a_in ? jc : ja;  // fluid end
    const int b = a_in ? ba : body[(long long)jc * (g.nx + 1) + ic];
    const double xi = node_x(g, ii), yi = node_y(g, ji);
    const double vx = node_x(g, io) - xi, vy = node_y(g, jo) - yi;
    const double t = cut_param(circ[b], xi, yi, vx, vy);
    pxy[2 * k] = xi + t * vx;
    pxy[2 * k + 1] = yi + t * vy;
    pbody[k] = (int8_t)b;
    pedge[k] = (int)e;
  }
}

// Displacement of an inside neighbour (in, jn) seen from a fluid node across edge e's
// cut point k: P - X_in.
__device__ __forceinline__ void cut_disp(const G& g, const double* __restrict__ pxy, int k, int in,
                                         int jn, double& dx, double& dy) {
  dx = pxy[2 * k] - node_x(g, in);
  dy = pxy[2 * k + 1] - node_y(g, jn);
}

// Up to MJS Jacobi sweeps in one launch (temporal blocking, as the bilinear mesh's
// k_jacobi_multi); the sweep of one fluid node off the domain's edge is
// d <- wx (d_E + d_W) + wy (d_N + d_S), an inside neighbour's d being its cut point's
// displacement P - I.  A block takes one displacement component of an MJT_X x MJT_Y tile of
// the last sweep's box, reads the tile widened by MJS nodes on every side into LDS and
// runs the sweeps there: after s sweeps the values are exact at least s nodes in from
// the region's edge.  A fluid node's inside neighbours contribute fixed values (their
// cut points' displacements), worked out once per launch into registers.  Every update
// is the single sweep's expression with the same operands in the same order, so the
// result is bit for bit that of the sweeps launched one by one.  Nodes outside a
// sweep's box have not changed since the start (the boxes only grow) and stay as they
// are.
constexpr int MJT_X = 64, MJT_Y = 16, MJS = 8;
struct MxBoxes {
  int i0[MJS], i1[MJS], j0[MJS], j1[MJS];
};

__global__ void __launch_bounds__(MB) k_mx_sweep_multi(G g, int ns, MxBoxes bx, double wx,
                                                       double wy,
                                                       const int8_t* __restrict__ body,
                                                       const int* __restrict__ hpt,
                                                       const int* __restrict__ vpt,
                                                       const double* __restrict__ pxy,
                                                       const double* __restrict__ src,
                                                       double* __restrict__ dst) {
  constexpr int RW = MJT_X + 2 * MJS, RH = MJT_Y + 2 * MJS;
  __shared__ double buf[2][RW * RH];
  __shared__ int8_t bd[RW * RH];  // node bodies (off the grid: -1)
  const long long nn = g.nn();
  const int comp = blockIdx.z;  // 0: x, 1: y
  const double* sv = src + comp * nn;
  double* dv = dst + comp * nn;
  const int last = ns - 1;
  const int gi0 = bx.i0[last] + (int)blockIdx.x * MJT_X - MJS;
  const int gj0 = bx.j0[last] + (int)blockIdx.y * MJT_Y - MJS;
  for (int e = threadIdx.x; e < RW * RH; e += MB) {
    const int i = gi0 + e % RW, j = gj0 + e / RW;
    const bool in = i >= 0 && i <= g.nx && j >= 0 && j <= g.ny;
    const long long n = (long long)j * (g.nx + 1) + i;
    buf[0][e] = in ? sv[n] : 0.0;
    bd[e] = in ? body[n] : (int8_t)-1;
  }
  __syncthreads();
  // per entry of this thread: updatable (a fluid node off the domain's edge), and the
  // fixed values of its inside neighbours (E, W, N, S; bit d of msk)
  static_assert(RW * RH % MB == 0, "whole region entries per thread");
  constexpr int NE = RW * RH / MB;
  int eli[NE], elj[NE], msk[NE];
  bool upd[NE];
  double fix[NE][4];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = (int)threadIdx.x + k * MB;
    eli[k] = e % RW;
    elj[k] = e / RW;
    const int i = gi0 + eli[k], j = gj0 + elj[k];
    // entries on the region's edge are never updated (their neighbours are not here)
    const bool inner = eli[k] > 0 && eli[k] < RW - 1 && elj[k] > 0 && elj[k] < RH - 1;
    const bool interior = i > 0 && i < g.nx && j > 0 && j < g.ny;
    upd[k] = inner && interior && bd[e] < 0;
    msk[k] = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) fix[k][d] = 0.0;
    if (upd[k]) {
      const int ne[4] = {e + 1, e - 1, e + RW, e - RW};
      const int ni[4] = {i + 1, i - 1, i, i}, nj[4] = {j, j, j + 1, j - 1};
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (bd[ne[d]] >= 0) {
          const int pk = d == 0   ? hpt[(long long)j * g.nx + i]
                         : d == 1 ? hpt[(long long)j * g.nx + i - 1]
                         : d == 2 ? vpt[(long long)j * (g.nx + 1) + i]
                                  : vpt[(long long)(j - 1) * (g.nx + 1) + i];
          double cx, cy;
          cut_disp(g, pxy, pk, ni[d], nj[d], cx, cy);
          fix[k][d] = comp ? cy : cx;
          msk[k] |= 1 << d;
        }
    }
  }
  int cur = 0;
  for (int sw = 0; sw < ns; ++sw) {
    const int li0 = max(bx.i0[sw] - gi0, sw + 1), li1 = min(bx.i1[sw] - gi0, RW - 2 - sw);
    const int lj0 = max(bx.j0[sw] - gj0, sw + 1), lj1 = min(bx.j1[sw] - gj0, RH - 2 - sw);
    const double* a = buf[cur];
    double* b = buf[cur ^ 1];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = (int)threadIdx.x + k * MB;
      double v = a[e];
      if (upd[k] && eli[k] >= li0 && eli[k] <= li1 && elj[k] >= lj0 && elj[k] <= lj1) {
        const double ve = (msk[k] & 1) ? fix[k][0] : a[e + 1];
        const double vw = (msk[k] & 2) ? fix[k][1] : a[e - 1];
        const double vn = (msk[k] & 4) ? fix[k][2] : a[e + RW];
        const double vs = (msk[k] & 8) ? fix[k][3] : a[e - RW];
        v = wx * (ve + vw) + wy * (vn + vs);
      }
      b[e] = v;
    }
    __syncthreads();
    cur ^= 1;
  }
  const int bi0 = bx.i0[last], bi1 = bx.i1[last], bj0 = bx.j0[last], bj1 = bx.j1[last];
  for (int e = threadIdx.x; e < MJT_X * MJT_Y; e += MB) {
    const int li = MJS + e % MJT_X, lj = MJS + e / MJT_X;
    const int i = gi0 + li, j = gj0 + lj;
    if (i >= bi0 && i <= bi1 && j >= bj0 && j <= bj1)
      dv[(long long)j * (g.nx + 1) + i] = buf[cur][lj * RW + li];
  }
}

// Cut point index of the edge from CCW corner k to corner k+1 of cell (i, j).
__device__ __forceinline__ int cell_edge_point(const G& g, const int* __restrict__ hpt,
                                               const int* __restrict__ vpt, int i, int j, int k) {
  if (k == 0) return hpt[(long long)j * g.nx + i];
  if (k == 1) return vpt[(long long)j * (g.nx + 1) + i + 1];
  if (k == 2) return hpt[(long long)(j + 1) * g.nx + i];
  return vpt[(long long)j * (g.nx + 1) + i];
}

// Elements of cell (i, j) (0, 1 or 2); with `out` non-null, their node lists.
__device__ int cell_elements(const G& g, const int8_t* __restrict__ body,
                             const int* __restrict__ hpt, const int* __restrict__ vpt,
                             const double* __restrict__ pxy, int i, int j, int* err,
                             int (*out)[4], int* nne) {
  const long long nn = g.nn();
  const long long c0 = (long long)j * (g.nx + 1) + i;
  const long long ids[4] = {c0, c0 + 1, c0 + g.nx + 2, c0 + g.nx + 1};
  int bb[4];
  bool ins[4];
  int nf = 0, bfirst = -1;
  bool two = false;
  for (int k = 0; k < 4; ++k) {
    bb[k] = body[ids[k]];
    ins[k] = bb[k] >= 0;
    if (!ins[k]) ++nf;
    if (ins[k]) {
      if (bfirst < 0) bfirst = bb[k];
      else if (bb[k] != bfirst) two = true;
    }
  }
  if (nf == 4) {
    if (out) {
      for (int k = 0; k < 4; ++k) out[0][k] = (int)ids[k];
      nne[0] = 4;
    }
    return 1;
  }
  if (two) {
    if (err) err[1] = 1;
    return 0;
  }
  if (nf == 0) return 0;
  int changes = 0;
  for (int k = 0; k < 4; ++k) changes += ins[k] != ins[(k + 1) & 3];
  const double hmax = g.hx > g.hy ? g.hx : g.hy;
  if (changes == 4) {
    // inside and fluid corners alternate (a thin part of the body crosses the cell):
    // a triangle at each fluid corner, in corner order, slivers dropped
    int m = 0;
    for (int k = 0; k < 4; ++k) {
      if (ins[k]) continue;
      const int qa = cell_edge_point(g, hpt, vpt, i, j, (k + 3) & 3);
      const int qb = cell_edge_point(g, hpt, vpt, i, j, k);
      const double gx = fabs(pxy[2 * qa] - pxy[2 * qb]);
      const double gy = fabs(pxy[2 * qa + 1] - pxy[2 * qb + 1]);
      const double gap = gx > gy ? gx : gy;
      if (!(gap >= SLIVER * hmax)) continue;
      if (out) {
        out[m][0] = (int)(nn + qa);
        out[m][1] = (int)ids[k];
        out[m][2] = (int)(nn + qb);
        out[m][3] = -1;
        nne[m] = 3;
      }
      ++m;
    }
    return m;
  }
  if (nf == 1) {
    // triangle: the fluid corner and the cut points on its two edges, CCW from corner 0
    int poly[3], np_ = 0;
    int pts[2], npt = 0;
    for (int k = 0; k < 4; ++k) {
      if (!ins[k]) poly[np_++] = (int)ids[k];
      if (ins[k] != ins[(k + 1) & 3]) {
        const int q = cell_edge_point(g, hpt, vpt, i, j, k);
        pts[npt++] = q;
        poly[np_++] = (int)(nn + q);
      }
    }
    const double gx = fabs(pxy[2 * pts[0]] - pxy[2 * pts[1]]);
    const double gy = fabs(pxy[2 * pts[0] + 1] - pxy[2 * pts[1] + 1]);
    const double gap = gx > gy ? gx : gy;
    if (!(gap >= SLIVER * hmax)) return 0;  // a sliver (max-norm gap below 1e-12 h)
    if (out) {
      for (int k = 0; k < 3; ++k) out[0][k] = poly[k];
      out[0][3] = -1;
      nne[0] = 3;
    }
    return 1;
  }
  if (nf == 2) {
    if (out) {
      int np_ = 0;
      for (int k = 0; k < 4; ++k) {
        if (!ins[k]) out[0][np_++] = (int)ids[k];
        if (ins[k] != ins[(k + 1) & 3])
          out[0][np_++] = (int)(nn + cell_edge_point(g, hpt, vpt, i, j, k));
      }
      nne[0] = 4;
    }
    return 1;
  }
  // pentagon: split at the cut point after the inside corner
  if (out) {
    int kin = 0;
    while (!ins[kin]) ++kin;
    const int pa = (int)(nn + cell_edge_point(g, hpt, vpt, i, j, kin));
    const int pb = (int)(nn + cell_edge_point(g, hpt, vpt, i, j, (kin + 3) & 3));
    const int c1 = (int)ids[(kin + 1) & 3], c2 = (int)ids[(kin + 2) & 3], c3 = (int)ids[(kin + 3) & 3];
    out[0][0] = pa;
    out[0][1] = c1;
    out[0][2] = c2;
    out[0][3] = -1;
    nne[0] = 3;
    out[1][0] = pa;
    out[1][1] = c2;
    out[1][2] = c3;
    out[1][3] = pb;
    nne[1] = 4;
  }
  return 2;
}

__global__ void k_mx_cell_count(G g, const int8_t* __restrict__ body, const int* __restrict__ hpt,
                                const int* __restrict__ vpt, const double* __restrict__ pxy,
                                int* __restrict__ cnt, int* __restrict__ err) {
  const long long nc = g.nc();
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc;
       c += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(c / g.nx), i = (int)(c - (long long)j * g.nx);
    cnt[c] = cell_elements(g, body, hpt, vpt, pxy, i, j, err, nullptr, nullptr);
  }
}

__global__ void k_mx_cells(G g, const int8_t* __restrict__ body, const int* __restrict__ hpt,
                           const int* __restrict__ vpt, const double* __restrict__ pxy,
                           const int* __restrict__ first, int* __restrict__ elem,
                           int8_t* __restrict__ nne, long long cap) {
  const long long nc = g.nc();
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc;
       c += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(c / g.nx), i = (int)(c - (long long)j * g.nx);
    int out[2][4];
    int nl[2];
    const int m = cell_elements(g, body, hpt, vpt, pxy, i, j, nullptr, out, nl);
    for (int q = 0; q < m; ++q) {
      const long long e = (long long)first[c] + q;
      if (e >= cap) break;
      for (int k = 0; k < 4; ++k) elem[4 * e + k] = out[q][k];
      nne[e] = (int8_t)nl[q];
    }
  }
}

// ---- element matrices and the apply ---------------------------------------------------
__device__ __forceinline__ void node_xy(const G& g, const double* __restrict__ disp,
                                        const double* __restrict__ pxy, long long n, double& x,
                                        double& y) {
  const long long nn = g.nn();
  if (n < nn) {
    const int j = (int)(n / (g.nx + 1)), i = (int)(n - (long long)j * (g.nx + 1));
    x = node_x(g, i) + disp[n];
    y = node_y(g, j) + disp[n + nn];
  } else {
    x = pxy[2 * (n - nn)];
    y = pxy[2 * (n - nn) + 1];
  }
}

}  // namespace mixed
}  // namespace mfp

#pragma clang fp contract(fast)

namespace mfp {
namespace mixed {

// K_e of element e, row-major 4 x 4 (triangles: leading 3 x 3, rest zero).
// Triangle (P1): K_ab = (b_a b_b + c_a c_b) / (4 A), b_a = y_(a+1) - y_(a+2),
// c_a = x_(a+2) - x_(a+1), 2A = sum b_a x_a.  Quadrilateral (Q1, 2x2 Gauss, points
// +-1/sqrt(3)): K_ab = sum_g det J (grad N_a . grad N_b).
__global__ void k_mx_kmat(G g, long long ne, const int* __restrict__ elem,
                          const int8_t* __restrict__ nne, const double* __restrict__ disp,
                          const double* __restrict__ pxy, double* __restrict__ K) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
       e += (long long)gridDim.x * blockDim.x) {
    double x[4], y[4];
    const int m = nne[e];
    for (int a = 0; a < m; ++a) node_xy(g, disp, pxy, elem[4 * e + a], x[a], y[a]);
    double k[16];
    for (int q = 0; q < 16; ++q) k[q] = 0.0;
    if (m == 3) {
      double b[3], c[3];
      for (int a = 0; a < 3; ++a) {
        const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
        b[a] = y[a1] - y[a2];
        c[a] = x[a2] - x[a1];
      }
      const double twoA = b[0] * x[0] + b[1] * x[1] + b[2] * x[2];
      const double s = 1.0 / (2.0 * twoA);
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) k[4 * a + d] = (b[a] * b[d] + c[a] * c[d]) * s;
    } else {
      const double xa[4] = {-1.0, 1.0, 1.0, -1.0}, ea[4] = {-1.0, -1.0, 1.0, 1.0};
      const double gp = 0.57735026918962576451;
      for (int q = 0; q < 4; ++q) {
        const double xi = xa[q] * gp, eta = ea[q] * gp;
        double dxi[4], deta[4];
        double j11 = 0, j12 = 0, j21 = 0, j22 = 0;
        for (int a = 0; a < 4; ++a) {
          dxi[a] = 0.25 * xa[a] * (1.0 + ea[a] * eta);
          deta[a] = 0.25 * ea[a] * (1.0 + xa[a] * xi);
          j11 += dxi[a] * x[a];
          j12 += dxi[a] * y[a];
          j21 += deta[a] * x[a];
          j22 += deta[a] * y[a];
        }
        const double det = j11 * j22 - j12 * j21;
        const double inv = 1.0 / det;
        double gx[4], gy[4];
        for (int a = 0; a < 4; ++a) {
          gx[a] = (j22 * dxi[a] - j12 * deta[a]) * inv;
          gy[a] = (-j21 * dxi[a] + j11 * deta[a]) * inv;
        }
        for (int a = 0; a < 4; ++a)
          for (int d = 0; d < 4; ++d) k[4 * a + d] += det * (gx[a] * gx[d] + gy[a] * gy[d]);
      }
    }
    for (int q = 0; q < 16; ++q) K[16 * e + q] = k[q];
  }
}

// Cells around mixed node n (up to four, in a fixed order; -1 when absent).
__device__ __forceinline__ void node_cells(const G& g, const int* __restrict__ pedge, long long n,
                                           long long (&cells)[4]) {
  const long long nn = g.nn();
  for (int k = 0; k < 4; ++k) cells[k] = -1;
  if (n < nn) {
    const int j = (int)(n / (g.nx + 1)), i = (int)(n - (long long)j * (g.nx + 1));
    int k = 0;
    for (int cj = j - 1; cj <= j; ++cj)
      for (int ci = i - 1; ci <= i; ++ci, ++k)
        if (ci >= 0 && cj >= 0 && ci < g.nx && cj < g.ny) cells[k] = (long long)cj * g.nx + ci;
  } else {
    const long long e = pedge[n - nn];
    int ia, ja, ic, jc;
    edge_ends(g, e, ia, ja, ic, jc);
    if (e < g.nh()) {  // horizontal edge: cells below and above
      if (ja - 1 >= 0) cells[0] = (long long)(ja - 1) * g.nx + ia;
      if (ja < g.ny) cells[1] = (long long)ja * g.nx + ia;
    } else {           // vertical edge: cells left and right
      if (ia - 1 >= 0) cells[0] = (long long)ja * g.nx + ia - 1;
      if (ia < g.nx) cells[1] = (long long)ja * g.nx + ia;
    }
  }
}

// Cell kinds for the product: no element (inside a body), the plain quadrilateral
// of a cell with four fluid corners (its six distinct off-diagonal entries stored),
// or a cut cell (its elements' full matrices read through the element lists).
enum : int8_t { CK_NONE = 0, CK_QUAD = 1, CK_CUT = 2 };

// Index of the off-diagonal entry (a, b) of a quadrilateral among its six.
__device__ __forceinline__ int pair_index(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo == 0 ? hi - 1 : lo == 1 ? hi + 1 : 5;
}

__global__ void k_mx_cellcoef(G g, const int8_t* __restrict__ body, const int* __restrict__ first,
                              const int* __restrict__ elem, const int8_t* __restrict__ nne,
                              const double* __restrict__ K, int8_t* __restrict__ ckind,
                              double* __restrict__ kc) {
  const long long nc = g.nc(), nn = g.nn();
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < nc;
       c += (long long)gridDim.x * blockDim.x) {
    const int e0 = first[c], e1 = first[c + 1];
    int8_t kind = CK_NONE;
    if (e1 - e0 == 1 && nne[e0] == 4 && elem[4 * e0] < nn && elem[4 * e0 + 1] < nn &&
        elem[4 * e0 + 2] < nn && elem[4 * e0 + 3] < nn)
      kind = CK_QUAD;
    else if (e1 > e0)
      kind = CK_CUT;
    ckind[c] = kind;
    double k[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (kind == CK_QUAD) {
      const double* ke = K + 16 * (long long)e0;
      k[0] = ke[1];
      k[1] = ke[2];
      k[2] = ke[3];
      k[3] = ke[6];
      k[4] = ke[7];
      k[5] = ke[11];
    } else if (kind == CK_CUT) {
      // the cell's matrix on its four corners: a cut point (value psi_b) goes to the
      // first inside corner, since every inside corner carries psi_b too
      const int j = (int)(c / g.nx), i = (int)(c - (long long)j * g.nx);
      const long long c0 = (long long)j * (g.nx + 1) + i;
      const long long ids[4] = {c0, c0 + 1, c0 + g.nx + 2, c0 + g.nx + 1};
      int kin = 0;
      while (kin < 3 && body[ids[kin]] < 0) ++kin;
      for (int e = e0; e < e1; ++e) {
        const int m = nne[e];
        int corner[4];
        for (int t = 0; t < m; ++t) {
          const long long id = elem[4 * e + t];
          int a = kin;
          for (int q = 0; q < 4; ++q)
            if (ids[q] == id) a = q;
          corner[t] = a;
        }
        const double* ke = K + 16 * (long long)e;
        for (int s = 0; s < m; ++s)
          for (int t = s + 1; t < m; ++t) {
            const int a = corner[s], b = corner[t];
            if (a != b) k[pair_index(a, b)] += ke[4 * s + t];
          }
      }
    }
    for (int q = 0; q < 6; ++q) kc[q * nc + c] = k[q];
  }
}

// Values of the vector K acts on (background nodes and cut points alike).
struct PlainVec {
  const double* p;
  __device__ __forceinline__ double bg(long long m) const { return p[m]; }
  __device__ __forceinline__ double cut(long long m) const { return p[m]; }
};
struct ApplyMx {
  G g;
  long long ntot;
  const int8_t* ckind;
  const double* kc;     // 6 nc, coefficient-major
  const int* first;
  const int* elem;
  const int8_t* nne;
  const double* K;
  const int* pedge;
};

// Row n of K v over the elements of cut cell c (the element's full matrix).
template <class V>
__device__ double cut_cell_row(const ApplyMx& a, long long c, long long n, const V& v) {
  const long long nn = a.g.nn();
  double acc = 0.0;
  for (int e = a.first[c]; e < a.first[c + 1]; ++e) {
    const int m = a.nne[e];
    int ids[4];
    int loc = -1;
    for (int t = 0; t < 4; ++t) {
      ids[t] = a.elem[4 * e + t];
      if (t < m && ids[t] == n) loc = t;
    }
    if (loc < 0) continue;
    const double* kr = a.K + 16 * (long long)e + 4 * loc;
    double s = 0.0;
    for (int t = 0; t < m; ++t) s += kr[t] * (ids[t] < nn ? v.bg(ids[t]) : v.cut(ids[t]));
    acc += s;
  }
  return acc;
}

// (K v)[n].  Background node (i, j): its four cells in the order (i-1, j-1), (i, j-1),
// (i-1, j), (i, j); a plain quadrilateral in difference form sum_b k_ab (v_b - v_a)
// (its rows sum to zero), a cut cell through its element lists.  Cut point: the two
// cells on either side of its edge.
template <class V>
__device__ __forceinline__ double apply_bg(const ApplyMx& a, long long n, int i, int j,
                                           double vn, const V& v);

template <class V>
__device__ __forceinline__ double apply_row(const ApplyMx& a, long long n, double vn,
                                            const V& v) {
  const G& g = a.g;
  const long long nn = g.nn();
  if (n >= nn) {
    long long cells[4];
    node_cells(g, a.pedge, n, cells);
    double acc = 0.0;
    for (int k = 0; k < 2; ++k)
      if (cells[k] >= 0 && a.ckind[cells[k]] == CK_CUT) acc += cut_cell_row(a, cells[k], n, v);
    return acc;
  }
  const int W = g.nx + 1;
  const int j = (int)(n / W), i = (int)(n - (long long)j * W);
  return apply_bg(a, n, i, j, vn, v);
}

// (K v)[n] at background node n = (i, j), as apply_row.
template <class V>
__device__ __forceinline__ double apply_bg(const ApplyMx& a, long long n, int i, int j,
                                           double vn, const V& v) {
  const G& g = a.g;
  const int W = g.nx + 1;
  const long long nc = g.nc();
  // Everything a plain cell needs is requested at once, at clamped addresses (a value
  // outside the grid belongs to a cell that is skipped): the 3 x 3 neighbourhood, the
  // four cells' kinds and the three entries of each cell's row of this node.  Tested
  // first, the kinds would put a second round trip before the entries.
  double P[3][3];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int ii = min(max(i + dx - 1, 0), g.nx), jj = min(max(j + dy - 1, 0), g.ny);
      P[dy][dx] = (dx == 1 && dy == 1) ? vn : v.bg((long long)jj * W + ii);
    }
  double acc = 0.0;
  bool cut = false;
  long long cc[4];
  // cell k = (i - 1 + (k & 1), j - 1 + (k >> 1)); the node is its corner ca (corners
  // CCW from the cell's (i, j)): 2, 3, 1, 0
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int ci = i - 1 + (k & 1), cj = j - 1 + (k >> 1);
    const bool in = ci >= 0 && cj >= 0 && ci < g.nx && cj < g.ny;
    const long long c =
        (long long)min(max(cj, 0), g.ny - 1) * g.nx + min(max(ci, 0), g.nx - 1);
    cc[k] = in ? c : -1;
    const int8_t kind = a.ckind[c];
    constexpr int CA[4] = {2, 3, 1, 0};
    const int ca = CA[k];
    const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b == ca) continue;
      const double vb = P[cj - j + 1 + cy[b]][ci - i + 1 + cx[b]];
      s += a.kc[pair_index(ca, b) * nc + c] * (vb - vn);
    }
    acc += (in && kind == CK_QUAD) ? s : 0.0;
    cut = cut || (in && kind == CK_CUT);
  }
  if (cut) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (cc[k] >= 0 && a.ckind[cc[k]] == CK_CUT) acc += cut_cell_row(a, cc[k], n, v);
  }
  return acc;
}

// Blocks [0, rows * bpr): background row j = block / bpr (a division per block, none per
// node), columns (block % bpr) MB + thread; the blocks after them: the cut points.
__global__ void __launch_bounds__(MB) k_mx_apply(ApplyMx a, int bpr, const double* __restrict__ p,
                                                 double* __restrict__ q) {
  const PlainVec v{p};
  const G& g = a.g;
  const int nbg = (g.ny + 1) * bpr;
  const int b = blockIdx.x;
  if (b < nbg) {
    const int j = b / bpr, i = (b - j * bpr) * MB + threadIdx.x;
    if (i > g.nx) return;
    const long long n = (long long)j * (g.nx + 1) + i;
    q[n] = apply_bg(a, n, i, j, p[n], v);
  } else {
    const long long n = g.nn() + (long long)(b - nbg) * MB + threadIdx.x;
    if (n < a.ntot) q[n] = apply_row(a, n, p[n], v);
  }
}

}  // namespace mixed
}  // namespace mfp

// ---- constrained solve on the mixed mesh ------------------------------------------------
// The constrained system A = T^T K T ties every cut point of body b to psi_b.  Every
// element lies in one background cell, and the inside corners of a cut cell are tied
// to the same psi_b, so T^T K T is also the sum over background cells of 4 x 4 corner
// matrices: a cut cell's elements condensed onto its corners (fluid corners keep their
// rows and columns, cut points are added to an inside corner).  The solve is then the
// one-kernel CG of the bilinear mesh reading those corner matrices as its stored
// element entries.
namespace mfp {
namespace mixed {

struct PsiB {
  double v[MFP_MAX_BODIES];
};

// psi at the mixed nodes from the solve's background values: inside nodes 0 (they are
// no mesh nodes), cut points psi_b.
__global__ void k_mx_psi_out(G g, long long npts, const int8_t* __restrict__ body,
                             const int8_t* __restrict__ pbody, PsiB pb, double* __restrict__ psi) {
  const long long nn = g.nn(), ntot = nn + npts;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < ntot;
       n += (long long)gridDim.x * blockDim.x) {
    if (n >= nn)
      psi[n] = pb.v[pbody[n - nn]];
    else if (body[n] >= 0)
      psi[n] = 0.0;
  }
}

// ---- host side ---------------------------------------------------------------------------
static G to_g(const mfp_grid& g) {
  G d;
  d.nx = g.nx;
  d.ny = g.ny;
  d.x0 = g.x0;
  d.y0 = g.y0;
  d.hx = grid_hx(g);
  d.hy = grid_hy(g);
  return d;
}

struct MeshWs {
  int* eflag;       // nh + nv
  int* eoff;        // nh + nv + 1
  int* ccnt;        // nc
  int* bsum;        // scan blocks + 1
  double* pxy;      // 2 (nh + nv)
  int8_t* pbody;    // nh + nv
  int* pedge;       // nh + nv
  int* elem;        // 4 * 2 nc
  int8_t* nne;      // 2 nc
  double* dtmp;     // 2 nn
  MxBody* circ;
  int* err;         // 4 flags
};

static size_t mesh_layout(const mfp_grid* gr, int nb, void* base, MeshWs* w) {
  Bump bp(base);
  const G g = to_g(*gr);
  const long long ne = g.nh() + g.nv(), nc = g.nc();
  MeshWs m{};
  m.eflag = bp.take<int>(ne);
  m.eoff = bp.take<int>(ne + 1);
  m.ccnt = bp.take<int>(nc);
  const long long mx = ne > nc ? ne : nc;
  m.bsum = bp.take<int>(scan_blocks(mx) + 2);
  m.pxy = bp.take<double>(2 * ne);
  m.pbody = bp.take<int8_t>(ne);
  m.pedge = bp.take<int>(ne);
  m.elem = bp.take<int>(8 * nc);
  m.nne = bp.take<int8_t>(2 * nc);
  m.dtmp = bp.take<double>(2 * g.nn());
  m.circ = bp.take<MxBody>(nb > 0 ? nb : 1);
  m.err = bp.take<int>(4);
  if (w) *w = m;
  return bp.off + 256;
}

}  // namespace mixed
}  // namespace mfp

using namespace mfp;
using namespace mfp::mixed;

extern "C" size_t mfp_mixed_workspace_size(const mfp_grid* grid, int32_t nbody) {
  if (!grid || grid->nx < 2 || grid->ny < 2 || nbody < 0 || nbody > MFP_MAX_BODIES) return 0;
  return mesh_layout(grid, nbody, nullptr, nullptr);
}

namespace mfp {
namespace mixed {

// A circle as a device body.
static MxBody circle_body(const mfp_circle& c) {
  MxBody b{};
  b.kind = MFP_BODY_CIRCLE;
  b.x = c.cx;
  b.y = c.cy;
  b.r = c.r;
  return b;
}

// A body description as a device body (cos and sin of the angle of attack from the C
// library), and a circle holding the whole body for the geometry checks: about the
// airfoil's placement point, the largest distance of 4097 boundary samples + 1%.
static int make_body(const mfp_body& d, MxBody* out, mfp_circle* bound) {
  if (d.kind == MFP_BODY_CIRCLE) {
    const mfp_circle c{d.x, d.y, d.r};
    *out = circle_body(c);
    *bound = c;
    return MFP_OK;
  }
  if (d.kind != MFP_BODY_JOUKOWSKI || !(d.r > 0.0) || !std::isfinite(d.x) ||
      !std::isfinite(d.y) || !std::isfinite(d.xi0) || !std::isfinite(d.eta0) ||
      !std::isfinite(d.alpha) || !(d.xi0 < 0.0) || d.xi0 < -d.r) {
    set_error("body: kind MFP_BODY_CIRCLE or MFP_BODY_JOUKOWSKI with c > 0, -c <= xi0 < 0 "
              "and finite parameters");
    return MFP_E_ARG;
  }
  MxBody b{};
  b.kind = MFP_BODY_JOUKOWSKI;
  b.x = d.x;
  b.y = d.y;
  b.r = d.r;
  b.xi0 = d.xi0;
  b.eta0 = d.eta0;
  b.c2 = d.r * d.r;
  b.R2 = (d.r - d.xi0) * (d.r - d.xi0) + d.eta0 * d.eta0;
  b.ca = std::cos(d.alpha);
  b.sa = std::sin(d.alpha);
  *out = b;
  const double R = std::sqrt(b.R2);
  double rmax = 0.0;
  for (int k = 0; k <= 4096; ++k) {
    const double th = 2.0 * M_PI * k / 4096.0;
    const double zr = d.xi0 + R * std::cos(th), zi = d.eta0 + R * std::sin(th);
    const double q = zr * zr + zi * zi;
    const double xr = zr + b.c2 * zr / q, xi = zi - b.c2 * zi / q;
    rmax = std::max(rmax, std::sqrt(xr * xr + xi * xi));
  }
  *bound = mfp_circle{d.x, d.y, rmax * 1.01};
  return MFP_OK;
}

static int mesh_impl(const mfp_grid* grid, const MxBody* bodies_h, const mfp_circle* bounds,
                     int32_t nbody, int32_t nsweeps, mfp_mixed_mesh_t* m, void* ws,
                     size_t ws_bytes, void* stream_) {
  // node box of every fluid node next to a cut edge: the bodies' bounding circles'
  // boxes widened by one node (empty when there is no body)
  int box[4] = {1, 0, 1, 0};
  {
    const double bhx = grid_hx(*grid), bhy = grid_hy(*grid);
    for (int b = 0; b < nbody; ++b) {
      const int i0 = (int)std::floor((bounds[b].cx - bounds[b].r - grid->x0) / bhx) - 1;
      const int i1 = (int)std::ceil((bounds[b].cx + bounds[b].r - grid->x0) / bhx) + 1;
      const int j0 = (int)std::floor((bounds[b].cy - bounds[b].r - grid->y0) / bhy) - 1;
      const int j1 = (int)std::ceil((bounds[b].cy + bounds[b].r - grid->y0) / bhy) + 1;
      if (b == 0 || box[0] > box[1]) {
        box[0] = i0;
        box[1] = i1;
        box[2] = j0;
        box[3] = j1;
      } else {
        box[0] = std::min(box[0], i0);
        box[1] = std::max(box[1], i1);
        box[2] = std::min(box[2], j0);
        box[3] = std::max(box[3], j1);
      }
    }
    box[0] = std::max(box[0], 0);
    box[2] = std::max(box[2], 0);
    box[1] = std::min(box[1], grid->nx);
    box[3] = std::min(box[3], grid->ny);
  }
  if (!m || !ws || !m->disp || !m->body || !m->hpt || !m->vpt || !m->cell_first ||
      nsweeps < 0 || m->cap_points < 0 || m->cap_elems < 0 ||
      (m->cap_points > 0 && (!m->pxy || !m->pbody || !m->pedge)) ||
      (m->cap_elems > 0 && (!m->elem || !m->nne))) {
    set_error("bad mesh arrays, capacities or nsweeps");
    return MFP_E_ARG;
  }
  const size_t need = mesh_layout(grid, nbody, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  MeshWs w;
  mesh_layout(grid, nbody, ws, &w);
  const G g = to_g(*grid);
  const long long nn = g.nn(), nh = g.nh(), ne = nh + g.nv(), nc = g.nc();
  if (nbody > 0)
    MFP_TRY_HIP(hipMemcpyAsync(w.circ, bodies_h, sizeof(MxBody) * nbody, hipMemcpyHostToDevice,
                               st));
  MFP_TRY_HIP(hipMemsetAsync(w.err, 0, 4 * sizeof(int), st));
  k_mx_classify<<<blocks_for(nn), MB, 0, st>>>(g, w.circ, nbody, m->body);
  k_mx_edge_flags<<<blocks_for(ne), MB, 0, st>>>(g, m->body, w.eflag, w.err);
  MFP_TRY_HIP(hipGetLastError());
  MFP_TRY(exclusive_scan(w.eflag, ne, w.bsum, w.eoff, st));
  k_mx_cut<<<blocks_for(ne), MB, 0, st>>>(g, w.circ, m->body, w.eflag, w.eoff, m->hpt, m->vpt,
                                          w.pxy, w.pbody, w.pedge, ne);
  MFP_TRY_HIP(hipGetLastError());
  // sweeps, ping-pong between the caller's array and the workspace
  MFP_TRY_HIP(hipMemsetAsync(m->disp, 0, sizeof(double) * 2 * nn, st));
  MFP_TRY_HIP(hipMemsetAsync(w.dtmp, 0, sizeof(double) * 2 * nn, st));
  const double hx = g.hx, hy = g.hy;
  const double s = 2.0 * (hx * hx + hy * hy);
  const double wx = (hy * hy) / s, wy = (hx * hx) / s;
  double* a = m->disp;
  double* b = w.dtmp;
  // a sizing call (no room for points or elements) needs no displacements
  const int sweeps = (m->cap_points == 0 && m->cap_elems == 0) || nbody == 0 ? 0 : nsweeps;
  // MJS sweeps per launch (k_mx_sweep_multi); sweep k covers box widened by k
  for (int k0 = 0; k0 < sweeps; k0 += MJS) {
    const int ns = std::min(MJS, sweeps - k0);
    MxBoxes bx;
    for (int q = 0; q < ns; ++q) {
      const int k = k0 + q;
      bx.i0[q] = std::max(0, box[0] - k);
      bx.i1[q] = std::min(g.nx, box[1] + k);
      bx.j0[q] = std::max(0, box[2] - k);
      bx.j1[q] = std::min(g.ny, box[3] + k);
    }
    const int lw = bx.i1[ns - 1] - bx.i0[ns - 1] + 1, lh = bx.j1[ns - 1] - bx.j0[ns - 1] + 1;
    if (lw > 0 && lh > 0) {
      const dim3 grid3((lw + MJT_X - 1) / MJT_X, (lh + MJT_Y - 1) / MJT_Y, 2);
      k_mx_sweep_multi<<<grid3, MB, 0, st>>>(g, ns, bx, wx, wy, m->body, m->hpt, m->vpt, w.pxy,
                                             a, b);
    }
    double* t = a;
    a = b;
    b = t;
  }
  MFP_TRY_HIP(hipGetLastError());
  if (a != m->disp)
    MFP_TRY_HIP(hipMemcpyAsync(m->disp, a, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
  k_mx_cell_count<<<blocks_for(nc), MB, 0, st>>>(g, m->body, m->hpt, m->vpt, w.pxy, w.ccnt, w.err);
  MFP_TRY_HIP(hipGetLastError());
  MFP_TRY(exclusive_scan(w.ccnt, nc, w.bsum, m->cell_first, st));
  k_mx_cells<<<blocks_for(nc), MB, 0, st>>>(g, m->body, m->hpt, m->vpt, w.pxy, m->cell_first,
                                            w.elem, w.nne, 2 * nc);
  MFP_TRY_HIP(hipGetLastError());
  int err[4];
  int counts[2];
  MFP_TRY_HIP(hipMemcpyAsync(err, w.err, sizeof(err), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipMemcpyAsync(&counts[0], w.eoff + ne, sizeof(int), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipMemcpyAsync(&counts[1], m->cell_first + nc, sizeof(int), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  if (err[0] || err[1]) {
    set_error(err[0] ? "a grid edge joins two bodies" : "a cell touches two bodies");
    return MFP_E_GEOMETRY;
  }
  m->n_points = counts[0];
  m->n_elems = counts[1];
  const long long np_ = counts[0] < m->cap_points ? counts[0] : m->cap_points;
  const long long nel = counts[1] < m->cap_elems ? counts[1] : m->cap_elems;
  if (np_ > 0) {
    MFP_TRY_HIP(hipMemcpyAsync(m->pxy, w.pxy, sizeof(double) * 2 * np_, hipMemcpyDeviceToDevice, st));
    MFP_TRY_HIP(hipMemcpyAsync(m->pbody, w.pbody, np_, hipMemcpyDeviceToDevice, st));
    MFP_TRY_HIP(hipMemcpyAsync(m->pedge, w.pedge, sizeof(int) * np_, hipMemcpyDeviceToDevice, st));
  }
  if (nel > 0) {
    MFP_TRY_HIP(hipMemcpyAsync(m->elem, w.elem, sizeof(int) * 4 * nel, hipMemcpyDeviceToDevice, st));
    MFP_TRY_HIP(hipMemcpyAsync(m->nne, w.nne, nel, hipMemcpyDeviceToDevice, st));
  }
  // triangles among the elements, and cut points per body
  std::vector<int8_t> hn((size_t)counts[1]);
  std::vector<int8_t> hp((size_t)counts[0]);
  if (counts[1] > 0)
    MFP_TRY_HIP(hipMemcpyAsync(hn.data(), w.nne, hn.size(), hipMemcpyDeviceToHost, st));
  if (counts[0] > 0)
    MFP_TRY_HIP(hipMemcpyAsync(hp.data(), w.pbody, hp.size(), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  long long ntri = 0;
  for (int8_t v : hn) ntri += v == 3;
  m->n_tri = ntri;
  std::vector<int> per((size_t)(nbody > 0 ? nbody : 1), 0);
  for (int8_t v : hp) ++per[v];
  for (int b = 0; b < nbody; ++b)
    if (per[b] == 0) {
      set_error("body %d holds no grid node: the grid does not resolve it", b);
      return MFP_E_GEOMETRY;
    }
  return MFP_OK;
}

}  // namespace mixed
}  // namespace mfp

extern "C" int mfp_mixed_mesh(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                              int32_t nsweeps, mfp_mixed_mesh_t* m, void* ws, size_t ws_bytes,
                              void* stream_) {
  clear_error();
  MFP_TRY(check_geometry(grid, circles_h, nbody));
  std::vector<MxBody> hb((size_t)(nbody > 0 ? nbody : 1));
  for (int b = 0; b < nbody; ++b) hb[b] = circle_body(circles_h[b]);
  return mesh_impl(grid, hb.data(), circles_h, nbody, nsweeps, m, ws, ws_bytes, stream_);
}

extern "C" int mfp_body_bounds(const mfp_body* bodies_h, int32_t nbody, mfp_circle* bounds_h) {
  clear_error();
  if (!bodies_h || !bounds_h || nbody < 0 || nbody > MFP_MAX_BODIES) {
    set_error("NULL argument or nbody outside [0, MFP_MAX_BODIES]");
    return MFP_E_ARG;
  }
  for (int b = 0; b < nbody; ++b) {
    MxBody tmp;
    MFP_TRY(make_body(bodies_h[b], &tmp, &bounds_h[b]));
  }
  return MFP_OK;
}

extern "C" int mfp_mixed_mesh_bodies(const mfp_grid* grid, const mfp_body* bodies_h,
                                     int32_t nbody, int32_t nsweeps, mfp_mixed_mesh_t* m,
                                     void* ws, size_t ws_bytes, void* stream_) {
  clear_error();
  if (nbody < 0 || nbody > MFP_MAX_BODIES || (nbody > 0 && !bodies_h)) {
    set_error("nbody outside [0, MFP_MAX_BODIES] or NULL bodies");
    return MFP_E_ARG;
  }
  std::vector<MxBody> hb((size_t)(nbody > 0 ? nbody : 1));
  std::vector<mfp_circle> bounds((size_t)(nbody > 0 ? nbody : 1));
  for (int b = 0; b < nbody; ++b) MFP_TRY(make_body(bodies_h[b], &hb[b], &bounds[b]));
  MFP_TRY(check_geometry(grid, bounds.data(), nbody));
  return mesh_impl(grid, hb.data(), bounds.data(), nbody, nsweeps, m, ws, ws_bytes, stream_);
}

namespace mfp {
namespace mixed {

struct SolveMx {
  double* K;       // 16 per element
  double* kc;      // 6 per cell, entry-major (corner matrices)
  int8_t* ckind;   // per cell
  void* solve_ws;  // the constrained solve's own workspace
  size_t solve_bytes;
};

static size_t solve_layout_mx(const G& g, long long nel, size_t solve_bytes, void* base,
                              SolveMx* out) {
  Bump bp(base);
  SolveMx s{};
  s.K = bp.take<double>(16 * (size_t)nel);
  s.kc = bp.take<double>(6 * (size_t)g.nc());
  s.ckind = bp.take<int8_t>(g.nc());
  s.solve_ws = bp.take<char>(solve_bytes);
  s.solve_bytes = solve_bytes;
  if (out) *out = s;
  return bp.off + 256;
}

static int check_mesh_arg(const mfp_grid* grid, const mfp_mixed_mesh_t* m) {
  MFP_TRY(check_grid(grid));
  if (!m || !m->disp || !m->body || !m->cell_first || m->n_points < 0 || m->n_elems < 0 ||
      m->n_points > m->cap_points || m->n_elems > m->cap_elems ||
      (m->n_points > 0 && (!m->pxy || !m->pbody || !m->pedge)) ||
      (m->n_elems > 0 && (!m->elem || !m->nne))) {
    set_error("mixed mesh arrays missing or counts above their capacities");
    return MFP_E_ARG;
  }
  return MFP_OK;
}

// Element matrices of every element, then the per-cell kinds and corner matrices;
// returns the product's arguments.
static ApplyMx setup_apply(const G& g, const mfp_mixed_mesh_t* m, const SolveMx& s,
                           hipStream_t st) {
  k_mx_kmat<<<blocks_for(m->n_elems), MB, 0, st>>>(g, m->n_elems, m->elem, m->nne, m->disp,
                                                     m->pxy, s.K);
  k_mx_cellcoef<<<blocks_for(g.nc()), MB, 0, st>>>(g, m->body, m->cell_first, m->elem, m->nne,
                                                   s.K, s.ckind, s.kc);
  ApplyMx a;
  a.g = g;
  a.ntot = g.nn() + m->n_points;
  a.ckind = s.ckind;
  a.kc = s.kc;
  a.first = m->cell_first;
  a.elem = m->elem;
  a.nne = m->nne;
  a.K = s.K;
  a.pedge = m->pedge;
  return a;
}

}  // namespace mixed
}  // namespace mfp

extern "C" size_t mfp_mixed_solve_workspace_size(const mfp_grid* grid, int64_t n_points,
                                                 int64_t n_elems, int32_t nbody,
                                                 const mfp_solver_opts* opts) {
  if (!grid || grid->nx < 2 || grid->ny < 2 || n_points < 0 || n_elems < 0 || nbody < 0 ||
      nbody > MFP_MAX_BODIES)
    return 0;
  const size_t sb = psi_solve_cells_workspace(grid, nbody, opts);
  if (sb == 0) return 0;
  return solve_layout_mx(to_g(*grid), n_elems, sb, nullptr, nullptr);
}

extern "C" int mfp_mixed_element_apply(const mfp_grid* grid, const mfp_mixed_mesh_t* m,
                                       const double* p, double* q, int32_t repeat,
                                       double* apply_ms_h, void* ws, size_t ws_bytes,
                                       void* stream_) {
  clear_error();
  MFP_TRY(check_mesh_arg(grid, m));
  if (!p || !q || !ws || repeat < 1) {
    set_error("NULL pointer or repeat < 1");
    return MFP_E_ARG;
  }
  const G g = to_g(*grid);
  const long long ntot = g.nn() + m->n_points;
  const size_t need = solve_layout_mx(g, m->n_elems, 0, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveMx s;
  solve_layout_mx(g, m->n_elems, 0, ws, &s);
  const ApplyMx a = setup_apply(g, m, s, st);
  MFP_TRY_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  MFP_TRY_HIP(hipEventCreate(&e0));
  MFP_TRY_HIP(hipEventCreate(&e1));
  MFP_TRY_HIP(hipEventRecord(e0, st));
  const int bpr = (grid->nx + 1 + MB - 1) / MB;
  const long long ncut = ntot - (long long)(grid->nx + 1) * (grid->ny + 1);
  const long long nblk = (long long)(grid->ny + 1) * bpr + (ncut + MB - 1) / MB;
  for (int k = 0; k < repeat; ++k) k_mx_apply<<<(unsigned)nblk, MB, 0, st>>>(a, bpr, p, q);
  MFP_TRY_HIP(hipEventRecord(e1, st));
  const hipError_t le = hipGetLastError();
  float ms = 0.f;
  hipError_t se = hipEventSynchronize(e1);
  if (se == hipSuccess) se = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (le != hipSuccess || se != hipSuccess) {
    set_error("mixed apply: %s", hipGetErrorString(le != hipSuccess ? le : se));
    return MFP_E_HIP;
  }
  if (apply_ms_h) *apply_ms_h = ms / repeat;
  return MFP_OK;
}

namespace mfp {
namespace mixed {

static int count_kutta(const double* kutta_xy_h, int nbody) {
  int nk = 0;
  if (kutta_xy_h)
    for (int b = 0; b < nbody; ++b)
      nk += !(std::isnan(kutta_xy_h[2 * b]) && std::isnan(kutta_xy_h[2 * b + 1]));
  return nk;
}

static size_t mixed_solve_bytes(const mfp_grid* grid, int nbody, int nk,
                                const mfp_solver_opts* opts, bool kutta) {
  return kutta ? psi_solve_cells_kutta_workspace(grid, nbody, nk, opts)
               : psi_solve_cells_workspace(grid, nbody, opts);
}

static int mixed_solve_impl(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                            const mfp_mixed_mesh_t* m, const mfp_flow* flow,
                            const mfp_solver_opts* opts, const double* kutta_xy_h,
                            int32_t pair_lo, int32_t pair_hi, double* psi, double* psi_b_h,
                            double* Q_h, double* copfi_h, int64_t* kutta_node_h,
                            mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream_) {
  MFP_TRY(check_geometry(grid, circles_h, nbody));
  MFP_TRY(check_mesh_arg(grid, m));
  if (!flow || !opts || !psi || !ws || (nbody > 0 && !psi_b_h)) {
    set_error("NULL argument");
    return MFP_E_ARG;
  }
  if (opts->psi0) {
    set_error("no warm start on the mixed mesh");
    return MFP_E_ARG;
  }
  const G g = to_g(*grid);
  const bool kutta = kutta_xy_h != nullptr;
  const int nk = count_kutta(kutta_xy_h, nbody);
  const size_t sb = mixed_solve_bytes(grid, nbody, nk, opts, kutta);
  if (sb == 0) {
    set_error("invalid solver options");
    return MFP_E_ARG;
  }
  const size_t need = solve_layout_mx(g, m->n_elems, sb, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  SolveMx s;
  solve_layout_mx(g, m->n_elems, sb, ws, &s);
  (void)setup_apply(g, m, s, st);
  MFP_TRY_HIP(hipGetLastError());
  // background-node values first (the mixed numbering starts with them)
  std::vector<double> pb((size_t)(nbody > 0 ? nbody : 1));
  const int rc = kutta ? psi_solve_cells_kutta(grid, circles_h, nbody, m->disp, m->body, s.kc,
                                               flow, opts, kutta_xy_h, pair_lo, pair_hi, psi,
                                               pb.data(), Q_h, copfi_h, kutta_node_h, stats_h,
                                               s.solve_ws, s.solve_bytes, st)
                       : psi_solve_cells(grid, circles_h, nbody, m->disp, m->body, s.kc, flow,
                                         opts, pair_lo, pair_hi, psi, pb.data(), Q_h, copfi_h,
                                         stats_h, s.solve_ws, s.solve_bytes, st);
  if (rc < 0) return rc;
  PsiB hb{};
  for (int b = 0; b < nbody; ++b) {
    hb.v[b] = pb[b];
    psi_b_h[b] = pb[b];
  }
  const long long ntot = g.nn() + m->n_points;
  k_mx_psi_out<<<blocks_for(ntot), MB, 0, st>>>(g, m->n_points, m->body, m->pbody, hb, psi);
  MFP_TRY_HIP(hipGetLastError());
  MFP_TRY_HIP(hipStreamSynchronize(st));
  return rc;
}

}  // namespace mixed
}  // namespace mfp

extern "C" int mfp_mixed_psi_solve(const mfp_grid* grid, const mfp_circle* circles_h,
                                   int32_t nbody, const mfp_mixed_mesh_t* m,
                                   const mfp_flow* flow, const mfp_solver_opts* opts,
                                   int32_t pair_lo, int32_t pair_hi, double* psi,
                                   double* psi_b_h, double* Q_h, double* copfi_h,
                                   mfp_stats* stats_h, void* ws, size_t ws_bytes,
                                   void* stream_) {
  clear_error();
  return mixed_solve_impl(grid, circles_h, nbody, m, flow, opts, nullptr, pair_lo, pair_hi, psi,
                          psi_b_h, Q_h, copfi_h, nullptr, stats_h, ws, ws_bytes, stream_);
}

extern "C" size_t mfp_mixed_kutta_workspace_size(const mfp_grid* grid, int64_t n_points,
                                                 int64_t n_elems, int32_t nbody, int32_t nkutta,
                                                 const mfp_solver_opts* opts) {
  if (!grid || grid->nx < 2 || grid->ny < 2 || n_points < 0 || n_elems < 0 || nbody < 0 ||
      nbody > MFP_MAX_BODIES || nkutta < 0 || nkutta > nbody)
    return 0;
  const size_t sb = psi_solve_cells_kutta_workspace(grid, nbody, nkutta, opts);
  if (sb == 0) return 0;
  return solve_layout_mx(to_g(*grid), n_elems, sb, nullptr, nullptr);
}

extern "C" int mfp_mixed_psi_solve_kutta(const mfp_grid* grid, const mfp_circle* circles_h,
                                         int32_t nbody, const mfp_mixed_mesh_t* m,
                                         const mfp_flow* flow, const mfp_solver_opts* opts,
                                         const double* kutta_xy_h, int32_t pair_lo,
                                         int32_t pair_hi, double* psi, double* psi_b_h,
                                         double* Q_h, double* copfi_h, int64_t* kutta_node_h,
                                         mfp_stats* stats_h, void* ws, size_t ws_bytes,
                                         void* stream_) {
  clear_error();
  if (!kutta_xy_h) {
    set_error("NULL Kutta points");
    return MFP_E_ARG;
  }
  return mixed_solve_impl(grid, circles_h, nbody, m, flow, opts, kutta_xy_h, pair_lo, pair_hi,
                          psi, psi_b_h, Q_h, copfi_h, kutta_node_h, stats_h, ws, ws_bytes,
                          stream_);
}
