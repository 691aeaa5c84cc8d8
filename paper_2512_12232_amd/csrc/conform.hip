// Body-conforming mesh on the GPU (section "Body-Conforming Grid Generation").
//
//   k_classify      node -> body id by the FP64 test (x-cx)^2 + (y-cy)^2 <= r^2
//   k_snap          body nodes with a fluid node among their eight neighbours are
//                   moved radially onto their circle (d_ik = x_ik - x_gk); others deep
//   k_jacobi_multi  up to 8 Jacobi sweeps d <- wx (d_E + d_W) + wy (d_N + d_S) of the
//                   displacement Laplace problem on fluid nodes off the outer boundary
//   k_tangle        Gauss-point Jacobian determinants of active cells must be > 0
//
// Every floating-point expression here is evaluated without contraction into fused
// multiply-adds, so the mesh is reproducible bit for bit and equals a plain IEEE
// evaluation of the same expressions in the same order.  Sweep k only touches the
// node box around the circles widened by k + 2 nodes: a Jacobi sweep moves
// information by one node per sweep, so every node outside that box still holds its
// initial value (zero), exactly as if the whole grid had been swept.
#include <cmath>

#include "mfp_internal.h"

#pragma clang fp contract(off)

namespace mfp {

struct GridD {
  int nx, ny;
  double x0, y0, hx, hy;
};

__global__ void k_classify(GridD g, const mfp_circle* __restrict__ circ, int nb,
                           int8_t* __restrict__ kind, int8_t* __restrict__ body) {
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn;
       n += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(n / (g.nx + 1));
    const int i = (int)(n - (long long)j * (g.nx + 1));
    const double x = g.x0 + (double)i * g.hx;
    const double y = g.y0 + (double)j * g.hy;
    int b_in = -1;
    for (int b = 0; b < nb; ++b) {
      const double dx = x - circ[b].cx;
      const double dy = y - circ[b].cy;
      if (dx * dx + dy * dy <= circ[b].r * circ[b].r) b_in = b;
    }
    body[n] = (int8_t)b_in;
    kind[n] = MFP_FLUID;
  }
}

__global__ void k_snap(GridD g, const mfp_circle* __restrict__ circ,
                       int8_t* __restrict__ kind, const int8_t* __restrict__ body,
                       double* __restrict__ disp) {
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn;
       n += (long long)gridDim.x * blockDim.x) {
    const int b = body[n];
    double ddx = 0.0, ddy = 0.0;
    if (b >= 0) {
      const int j = (int)(n / (g.nx + 1));
      const int i = (int)(n - (long long)j * (g.nx + 1));
      bool near_fluid = false;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int ii = i + di, jj = j + dj;
          if (ii >= 0 && ii <= g.nx && jj >= 0 && jj <= g.ny &&
              body[(long long)jj * (g.nx + 1) + ii] < 0)
            near_fluid = true;
        }
      kind[n] = near_fluid ? MFP_SNAPPED : MFP_DEEP;
      if (near_fluid) {
        const double x = g.x0 + (double)i * g.hx;
        const double y = g.y0 + (double)j * g.hy;
        const double cx = circ[b].cx, cy = circ[b].cy, r = circ[b].r;
        const double dx = x - cx;
        const double dy = y - cy;
        const double rho = __builtin_sqrt(dx * dx + dy * dy);
        const double s = r / rho;
        const double px = cx + s * dx;
        const double py = cy + s * dy;
        ddx = px - x;
        ddy = py - y;
      }
    }
    disp[n] = ddx;
    disp[n + nn] = ddy;
  }
}

// Up to JS Jacobi sweeps in one launch (temporal blocking).  A block takes one
// displacement component of a JT_X x JT_Y tile of the last sweep's box, reads the tile
// widened by JS nodes on every side into LDS, and runs the sweeps there: after s sweeps
// the values are exact at least s nodes in from the region's edge, so the tile itself
// is exact after JS.  Sweep s updates exactly the nodes the single sweep would (fluid
// nodes in that sweep's box) with the same expression in the same order, so the
// result is bit for bit that of the sweeps launched one by one.  Nodes outside a
// sweep's box have not changed since the start (the boxes only grow) and are left as
// they are, in LDS and in both global buffers.
constexpr int JT_X = 64, JT_Y = 16, JS = 8;
struct SweepBoxes {
  int i0[JS], i1[JS], j0[JS], j1[JS];
};

__global__ void __launch_bounds__(BLOCK) k_jacobi_multi(int nx, int ny, int ns, SweepBoxes bx,
                                                        double wx, double wy,
                                                        const int8_t* __restrict__ kind,
                                                        const double* __restrict__ src,
                                                        double* __restrict__ dst) {
  constexpr int RW = JT_X + 2 * JS, RH = JT_Y + 2 * JS;
  __shared__ double buf[2][RW * RH];
  __shared__ int8_t kd[RW * RH];
  const long long nn = (long long)(nx + 1) * (ny + 1);
  const double* s = src + blockIdx.z * nn;
  double* d = dst + blockIdx.z * nn;
  const int last = ns - 1;
  // region origin: tiles start at the last box's corner
  const int gi0 = bx.i0[last] + (int)blockIdx.x * JT_X - JS;
  const int gj0 = bx.j0[last] + (int)blockIdx.y * JT_Y - JS;
  for (int e = threadIdx.x; e < RW * RH; e += BLOCK) {
    const int i = gi0 + e % RW, j = gj0 + e / RW;
    const bool in = i >= 0 && i <= nx && j >= 0 && j <= ny;
    const long long n = (long long)j * (nx + 1) + i;
    buf[0][e] = in ? s[n] : 0.0;
    kd[e] = in ? kind[n] : (int8_t)-1;  // off the grid: never updated, never read by an update
  }
  __syncthreads();
  // each thread keeps the same NE region entries in every sweep: their coordinates and
  // node kinds are worked out once
  static_assert(RW * RH % BLOCK == 0, "whole region entries per thread");
  constexpr int NE = RW * RH / BLOCK;
  int eli[NE], elj[NE];
  bool efl[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = (int)threadIdx.x + k * BLOCK;
    eli[k] = e % RW;
    elj[k] = e / RW;
    efl[k] = kd[e] == MFP_FLUID;
  }
  int cur = 0;
  for (int sw = 0; sw < ns; ++sw) {
    // box of sweep sw in region coordinates, cut to the entries it can update
    const int li0 = max(bx.i0[sw] - gi0, sw + 1), li1 = min(bx.i1[sw] - gi0, RW - 2 - sw);
    const int lj0 = max(bx.j0[sw] - gj0, sw + 1), lj1 = min(bx.j1[sw] - gj0, RH - 2 - sw);
    const double* a = buf[cur];
    double* b = buf[cur ^ 1];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = (int)threadIdx.x + k * BLOCK;
      double v = a[e];
      if (efl[k] && eli[k] >= li0 && eli[k] <= li1 && elj[k] >= lj0 && elj[k] <= lj1)
        v = wx * (a[e + 1] + a[e - 1]) + wy * (a[e + RW] + a[e - RW]);
      b[e] = v;
    }
    __syncthreads();
    cur ^= 1;
  }
  const int bi0 = bx.i0[last], bi1 = bx.i1[last], bj0 = bx.j0[last], bj1 = bx.j1[last];
  for (int e = threadIdx.x; e < JT_X * JT_Y; e += BLOCK) {
    const int li = JS + e % JT_X, lj = JS + e / JT_X;
    const int i = gi0 + li, j = gj0 + lj;
    if (i >= bi0 && i <= bi1 && j >= bj0 && j <= bj1)
      d[(long long)j * (nx + 1) + i] = buf[cur][lj * RW + li];
  }
}

// Jacobian determinants at the four Gauss points of every active cell in the box.
__global__ void k_tangle(GridD g, int ci0, int cj0, int bw, int bh,
                         const int8_t* __restrict__ body, const double* __restrict__ disp,
                         int* __restrict__ bad) {
  const int ci = ci0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int cj = cj0 + (int)blockIdx.y;
  if (ci >= ci0 + bw || (int)blockIdx.y >= bh) return;
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  const long long n0 = (long long)cj * (g.nx + 1) + ci;
  const long long nd[4] = {n0, n0 + 1, n0 + g.nx + 2, n0 + g.nx + 1};
  const int b0 = body[nd[0]];
  if (b0 >= 0 && body[nd[1]] == b0 && body[nd[2]] == b0 && body[nd[3]] == b0) return;
  const double bx[4] = {0.0, g.hx, g.hx, 0.0}, by[4] = {0.0, 0.0, g.hy, g.hy};
  double x[4], y[4];
  for (int a = 0; a < 4; ++a) {
    x[a] = bx[a] + disp[nd[a]];
    y[a] = by[a] + disp[nd[a] + nn];
  }
  const double s = 0.57735026918962576451;
  const double xi_a[4] = {-1, 1, 1, -1}, eta_a[4] = {-1, -1, 1, 1};
  for (int q = 0; q < 4; ++q) {
    const double xi = xi_a[q] * s, eta = eta_a[q] * s;
    double j11 = 0, j12 = 0, j21 = 0, j22 = 0;
    for (int a = 0; a < 4; ++a) {
      const double nxi = 0.25 * xi_a[a] * (1.0 + eta_a[a] * eta);
      const double neta = 0.25 * eta_a[a] * (1.0 + xi_a[a] * xi);
      j11 += nxi * x[a];
      j12 += nxi * y[a];
      j21 += neta * x[a];
      j22 += neta * y[a];
    }
    if (!(j11 * j22 - j12 * j21 > 0.0)) atomicOr(bad, 1);
  }
}

static GridD to_dev(const mfp_grid& g) {
  return GridD{g.nx, g.ny, g.x0, g.y0, grid_hx(g), grid_hy(g)};
}

// Union of the circles' node boxes widened by `pad`, clipped to [lo, hi].
static Box union_box(const mfp_grid& g, const mfp_circle* c, int nb, int pad, int ilo,
                     int ihi, int jlo, int jhi) {
  Box u{1, 0, 1, 0};
  bool first = true;
  for (int b = 0; b < nb; ++b) {
    Box x = circle_box(g, c[b], pad, ilo, ihi, jlo, jhi);
    if (x.empty()) continue;
    if (first) {
      u = x;
      first = false;
    } else {
      u.i0 = x.i0 < u.i0 ? x.i0 : u.i0;
      u.j0 = x.j0 < u.j0 ? x.j0 : u.j0;
      u.i1 = x.i1 > u.i1 ? x.i1 : u.i1;
      u.j1 = x.j1 > u.j1 ? x.j1 : u.j1;
    }
  }
  return u;
}

// Transposed Jacobi sweep (adjoint of one sweep of k_jacobi_multi): with upd(n) = fluid node off
// the outer boundary, g_new[m] = [m fixed] g[m] + sum over update neighbours n of
// w(n, m) g[n].
__global__ void k_jacobi_sweep_T(int nx, int ny, int i0, int j0, int bw, int bh, double wx,
                                 double wy, const int8_t* __restrict__ kind,
                                 const double* __restrict__ src, double* __restrict__ dst) {
  const long long nn = (long long)(nx + 1) * (ny + 1);
  const int i = i0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int j = j0 + (int)blockIdx.y;
  if (i >= i0 + bw || (int)blockIdx.y >= bh) return;
  const long long n = (long long)j * (nx + 1) + i;
  auto upd = [&](int ii, int jj) {
    return ii >= 1 && ii <= nx - 1 && jj >= 1 && jj <= ny - 1 &&
           kind[(long long)jj * (nx + 1) + ii] == MFP_FLUID;
  };
  const bool ue = upd(i + 1, j), uw = upd(i - 1, j), un = upd(i, j + 1), us = upd(i, j - 1);
  const bool self = upd(i, j);
  for (int c = 0; c < 2; ++c) {
    const double* s = src + c * nn;
    const double ge = ue ? s[n + 1] : 0.0, gw = uw ? s[n - 1] : 0.0;
    const double gn = un ? s[n + nx + 1] : 0.0, gs = us ? s[n - nx - 1] : 0.0;
    dst[n + c * nn] = (self ? 0.0 : s[n]) + (wx * (ge + gw) + wy * (gn + gs));
  }
}

// One block per body: derivatives of the snapped displacements d0 = c + (r/rho)(x - c) - x
// with respect to the centre (I - (r/rho)(I - u u^T), u = (x - c)/rho) and the radius
// (u), applied to the incoming gradient and summed over the body's snapped nodes.
__global__ void __launch_bounds__(BLOCK) k_project_grad(GridD g, const mfp_circle* __restrict__ circ,
                                                        const int* __restrict__ boxes,
                                                        const int8_t* __restrict__ kind,
                                                        const int8_t* __restrict__ body,
                                                        const double* __restrict__ gd,
                                                        double* __restrict__ out) {
  __shared__ double s_red[3][BLOCK / 64];
  const int b = blockIdx.x;
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  const int i0 = boxes[4 * b], i1 = boxes[4 * b + 1], j0 = boxes[4 * b + 2], j1 = boxes[4 * b + 3];
  const int bw = i1 - i0 + 1;
  const long long total = (i1 >= i0 && j1 >= j0) ? (long long)bw * (j1 - j0 + 1) : 0;
  const double cx = circ[b].cx, cy = circ[b].cy, r = circ[b].r;
  double acx = 0.0, acy = 0.0, ar = 0.0;
  for (long long e = threadIdx.x; e < total; e += BLOCK) {
    const int i = i0 + (int)(e % bw), j = j0 + (int)(e / bw);
    const long long n = (long long)j * (g.nx + 1) + i;
    if (kind[n] != MFP_SNAPPED || body[n] != b) continue;
    const double dx = (g.x0 + (double)i * g.hx) - cx, dy = (g.y0 + (double)j * g.hy) - cy;
    const double rho = sqrt(dx * dx + dy * dy);
    const double ux = dx / rho, uy = dy / rho, f = r / rho;
    const double gx = gd[n], gy = gd[n + nn];
    acx += (1.0 - f * (1.0 - ux * ux)) * gx + f * ux * uy * gy;
    acy += f * ux * uy * gx + (1.0 - f * (1.0 - uy * uy)) * gy;
    ar += ux * gx + uy * gy;
  }
  double v[3] = {acx, acy, ar};
  for (int k = 0; k < 3; ++k) {
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0) s_red[k][threadIdx.x >> 6] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    out[3 * b + k] = (s_red[k][0] + s_red[k][1]) + (s_red[k][2] + s_red[k][3]);
  }
}

struct ConformWs {
  mfp_circle* circ;
  double* tmp;  // second displacement buffer
  int* flag;
};

static size_t conform_layout(const mfp_grid* g, int nb, void* ws, ConformWs* out) {
  Bump bp(ws);
  const size_t nn = (size_t)(g->nx + 1) * (g->ny + 1);
  ConformWs w;
  w.circ = bp.take<mfp_circle>(nb > 0 ? nb : 1);
  w.tmp = bp.take<double>(2 * nn);
  w.flag = bp.take<int>(64);
  if (out) *out = w;
  return bp.off + 256;
}

}  // namespace mfp

using namespace mfp;

extern "C" size_t mfp_conform_workspace_size(const mfp_grid* grid, int32_t nbody) {
  if (!grid || grid->nx < 2 || grid->ny < 2) return 0;
  return conform_layout(grid, nbody, nullptr, nullptr);
}

extern "C" int mfp_mesh_conform(const mfp_grid* grid, const mfp_circle* circles_h,
                                int32_t nbody, int32_t nsweeps, double* disp, int8_t* kind,
                                int8_t* body, void* ws, size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_geometry(grid, circles_h, nbody));
  if (nsweeps < 0) {
    set_error("nsweeps < 0");
    return MFP_E_ARG;
  }
  if (!disp || !kind || !body || !ws) {
    set_error("NULL output or workspace pointer");
    return MFP_E_ARG;
  }
  const size_t need = conform_layout(grid, nbody, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  ConformWs w;
  conform_layout(grid, nbody, ws, &w);
  const mfp_grid& g = *grid;
  const GridD gd = to_dev(g);
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  if (nbody > 0)
    MFP_TRY_HIP(hipMemcpyAsync(w.circ, circles_h, sizeof(mfp_circle) * nbody,
                               hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemsetAsync(w.flag, 0, sizeof(int), st));
  const int nblk = (int)((nn + BLOCK - 1) / BLOCK < 65536 ? (nn + BLOCK - 1) / BLOCK : 65536);
  k_classify<<<nblk, BLOCK, 0, st>>>(gd, w.circ, nbody, kind, body);
  MFP_TRY_HIP(hipGetLastError());
  k_snap<<<nblk, BLOCK, 0, st>>>(gd, w.circ, kind, body, disp);
  MFP_TRY_HIP(hipGetLastError());

  const double hx = gd.hx, hy = gd.hy;
  const double s = 2.0 * (hx * hx + hy * hy);
  const double wx = (hy * hy) / s, wy = (hx * hx) / s;
  if (nsweeps > 0 && nbody > 0) {
    MFP_TRY_HIP(hipMemcpyAsync(w.tmp, disp, sizeof(double) * 2 * nn,
                               hipMemcpyDeviceToDevice, st));
    double* a = disp;
    double* b = w.tmp;
    // sweep k updates the fluid nodes of the circles' box widened by k + 1 nodes;
    // up to JS sweeps per launch
    for (int k = 1; k <= nsweeps;) {
      SweepBoxes sb;
      int ns = 0;
      while (ns < JS && k + ns <= nsweeps) {
        const Box bx = union_box(g, circles_h, nbody, k + ns + 1, 1, g.nx - 1, 1, g.ny - 1);
        if (bx.empty()) break;
        sb.i0[ns] = bx.i0;
        sb.i1[ns] = bx.i1;
        sb.j0[ns] = bx.j0;
        sb.j1[ns] = bx.j1;
        ++ns;
      }
      if (ns == 0) {  // nothing to sweep (cannot happen for accepted geometry)
        ++k;
        continue;
      }
      const int bw = sb.i1[ns - 1] - sb.i0[ns - 1] + 1, bh = sb.j1[ns - 1] - sb.j0[ns - 1] + 1;
      dim3 grd((bw + JT_X - 1) / JT_X, (bh + JT_Y - 1) / JT_Y, 2);
      k_jacobi_multi<<<grd, BLOCK, 0, st>>>(g.nx, g.ny, ns, sb, wx, wy, kind, a, b);
      MFP_TRY_HIP(hipGetLastError());
      double* t = a;
      a = b;
      b = t;
      k += ns;
    }
    if (a != disp)
      MFP_TRY_HIP(hipMemcpyAsync(disp, a, sizeof(double) * 2 * nn,
                                 hipMemcpyDeviceToDevice, st));
  }
  if (nbody > 0) {
    // cells whose nodes may have moved: the sweep box plus one cell
    const Box cb = union_box(g, circles_h, nbody, nsweeps + 3, 0, g.nx - 1, 0, g.ny - 1);
    if (!cb.empty()) {
      const int bw = cb.i1 - cb.i0 + 1, bh = cb.j1 - cb.j0 + 1;
      dim3 grd((bw + BLOCK - 1) / BLOCK, bh);
      k_tangle<<<grd, BLOCK, 0, st>>>(gd, cb.i0, cb.j0, bw, bh, body, disp, w.flag);
      MFP_TRY_HIP(hipGetLastError());
    }
  }
  int bad = 0;
  MFP_TRY_HIP(hipMemcpyAsync(&bad, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  if (bad) {
    set_error("tangled mesh: an active cell has a non-positive Jacobian determinant");
    return MFP_E_TANGLED;
  }
  return MFP_OK;
}

extern "C" size_t mfp_conform_grad_workspace_size(const mfp_grid* grid, int32_t nbody) {
  if (!grid || grid->nx < 2 || grid->ny < 2) return 0;
  Bump bp(nullptr);
  const size_t nn = (size_t)(grid->nx + 1) * (grid->ny + 1);
  bp.take<double>(2 * nn);
  bp.take<double>(2 * nn);
  bp.take<mfp_circle>(nbody > 0 ? nbody : 1);
  bp.take<int>(4 * (nbody > 0 ? nbody : 1));
  bp.take<double>(3 * (nbody > 0 ? nbody : 1));
  return bp.off + 256;
}

extern "C" int mfp_mesh_conform_grad(const mfp_grid* grid, const mfp_circle* circles_h,
                                     int32_t nbody, int32_t nsweeps, const int8_t* kind,
                                     const int8_t* body, const double* dL_ddisp,
                                     double* dL_dcentre_h, double* dL_dradius_h, void* ws,
                                     size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_geometry(grid, circles_h, nbody));
  if (nsweeps < 0 || !kind || !body || !dL_ddisp || !ws || (nbody > 0 && !dL_dcentre_h)) {
    set_error("bad argument");
    return MFP_E_ARG;
  }
  const size_t need = mfp_conform_grad_workspace_size(grid, nbody);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  if (nbody == 0) return MFP_OK;
  hipStream_t st = static_cast<hipStream_t>(stream_);
  const mfp_grid& g = *grid;
  const GridD gd = to_dev(g);
  const long long nn = (long long)(g.nx + 1) * (g.ny + 1);
  Bump bp(ws);
  double* A = bp.take<double>(2 * nn);
  double* B = bp.take<double>(2 * nn);
  mfp_circle* circ = bp.take<mfp_circle>(nbody);
  int* boxes = bp.take<int>(4 * nbody);
  double* out = bp.take<double>(3 * nbody);
  int hbox[4 * MFP_MAX_BODIES];
  for (int b = 0; b < nbody; ++b) {
    const Box x = circle_box(g, circles_h[b], 1, 0, g.nx, 0, g.ny);
    hbox[4 * b] = x.i0;
    hbox[4 * b + 1] = x.i1;
    hbox[4 * b + 2] = x.j0;
    hbox[4 * b + 3] = x.j1;
  }
  MFP_TRY_HIP(hipMemcpyAsync(circ, circles_h, sizeof(mfp_circle) * nbody, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(boxes, hbox, sizeof(int) * 4 * nbody, hipMemcpyHostToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(A, dL_ddisp, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
  MFP_TRY_HIP(hipMemcpyAsync(B, dL_ddisp, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
  const double hx = gd.hx, hy = gd.hy;
  const double sw = 2.0 * (hx * hx + hy * hy);
  const double wx = (hy * hy) / sw, wy = (hx * hx) / sw;
  // Transposed sweep s only needs nodes within nsweeps - s of a snapped node (the
  // snapped values after the last sweep are all that is read).
  double* a = A;
  double* b = B;
  for (int s = 1; s <= nsweeps; ++s) {
    const Box bx = union_box(g, circles_h, nbody, nsweeps - s + 2, 1, g.nx - 1, 1, g.ny - 1);
    if (!bx.empty()) {
      const int bw = bx.i1 - bx.i0 + 1, bh = bx.j1 - bx.j0 + 1;
      dim3 grd((bw + BLOCK - 1) / BLOCK, bh);
      k_jacobi_sweep_T<<<grd, BLOCK, 0, st>>>(g.nx, g.ny, bx.i0, bx.j0, bw, bh, wx, wy, kind, a, b);
      MFP_TRY_HIP(hipGetLastError());
    }
    double* t = a;
    a = b;
    b = t;
  }
  k_project_grad<<<nbody, BLOCK, 0, st>>>(gd, circ, boxes, kind, body, a, out);
  MFP_TRY_HIP(hipGetLastError());
  double hout[3 * MFP_MAX_BODIES];
  MFP_TRY_HIP(hipMemcpyAsync(hout, out, sizeof(double) * 3 * nbody, hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nbody; ++k) {
    dL_dcentre_h[2 * k] += hout[3 * k];
    dL_dcentre_h[2 * k + 1] += hout[3 * k + 1];
    if (dL_dradius_h) dL_dradius_h[k] += hout[3 * k + 2];
  }
  return MFP_OK;
}
