// Post-processing of a gap-ratio sweep (section "Effect of Gap Ratio"): the cubic
// least-squares fit of CoPFI over delta with its R^2 and mean square error.  A few
// hundred host values at most, so host code: Householder QR of the n x 4 matrix
// [x^3 x^2 x 1], then back substitution.
#include <cmath>
#include <vector>

#include "mfp_internal.h"

using namespace mfp;

extern "C" int mfp_cubic_fit(const double* x_h, const double* y_h, int32_t n, double* coef_h,
                             double* r2_h, double* mse_h) {
  clear_error();
  if (!x_h || !y_h || !coef_h) {
    set_error("NULL argument");
    return MFP_E_ARG;
  }
  if (n < 4) {
    set_error("a cubic fit needs at least 4 points (got %d)", n);
    return MFP_E_ARG;
  }
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x_h[i]) || !std::isfinite(y_h[i])) {
      set_error("non-finite value at %d", i);
      return MFP_E_ARG;
    }
  // A (column-major, n x 4) and the right-hand side
  std::vector<double> A(4 * (size_t)n), b(y_h, y_h + n);
  for (int i = 0; i < n; ++i) {
    const double x = x_h[i];
    A[i] = x * x * x;
    A[n + i] = x * x;
    A[2 * (size_t)n + i] = x;
    A[3 * (size_t)n + i] = 1.0;
  }
  double R[4][4] = {};
  for (int k = 0; k < 4; ++k) {
    double* a = &A[(size_t)k * n];
    double nrm = 0.0;
    for (int i = k; i < n; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    double scale = 0.0;
    for (int c = 0; c < 4; ++c) {
      const double* ac = &A[(size_t)c * n];
      for (int i = 0; i < n; ++i) scale = std::fmax(scale, std::fabs(ac[i]));
    }
    if (!(nrm > 1e-13 * scale * std::sqrt((double)n))) {
      set_error("x has fewer than 4 distinct values (rank-deficient fit)");
      return MFP_E_ARG;
    }
    // Householder vector v = a_k.. + sign(a_kk) |a| e_k, stored in place
    const double alpha = a[k] >= 0.0 ? -nrm : nrm;
    a[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < n; ++i) vv += a[i] * a[i];
    // apply H = I - 2 v v^T / (v^T v) to the later columns and to b
    for (int c = k + 1; c < 4; ++c) {
      double* ac = &A[(size_t)c * n];
      double d = 0.0;
      for (int i = k; i < n; ++i) d += a[i] * ac[i];
      const double f = 2.0 * d / vv;
      for (int i = k; i < n; ++i) ac[i] -= f * a[i];
    }
    double d = 0.0;
    for (int i = k; i < n; ++i) d += a[i] * b[i];
    const double f = 2.0 * d / vv;
    for (int i = k; i < n; ++i) b[i] -= f * a[i];
    R[k][k] = alpha;
    for (int c = k + 1; c < 4; ++c) R[k][c] = A[(size_t)c * n + k];
  }
  double c[4];
  for (int k = 3; k >= 0; --k) {
    double s = b[k];
    for (int m = k + 1; m < 4; ++m) s -= R[k][m] * c[m];
    c[k] = s / R[k][k];
  }
  double mean = 0.0;
  for (int i = 0; i < n; ++i) mean += y_h[i];
  mean /= n;
  double ss_res = 0.0, ss_tot = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = x_h[i];
    const double r = y_h[i] - (((c[0] * x + c[1]) * x + c[2]) * x + c[3]);
    ss_res += r * r;
    ss_tot += (y_h[i] - mean) * (y_h[i] - mean);
  }
  for (int k = 0; k < 4; ++k) coef_h[k] = c[k];
  if (r2_h) *r2_h = ss_tot > 0.0 ? 1.0 - ss_res / ss_tot : 1.0;
  if (mse_h) *mse_h = ss_res / n;
  return MFP_OK;
}

// ---------------------------------------------------------------------------------
// Contour lines of a nodal field on the conformed mesh: the flow net (contours of psi
// and phi, section "Governing Equation") and the stagnation streamlines psi = psi_b
// of section "Effect of Gap Ratio".  Marching squares over the active cells in the
// displaced node coordinates: a node is above the level when its value is >= the
// level; on each edge a -> b (0-1, 1-2, 2-3, 3-0) whose nodes differ the crossing is
// x_a + t (x_b - x_a), t = (level - f_a) / (f_b - f_a); two crossings give one segment
// (lower edge first), four (a saddle) two, paired by the mean of the four values (on
// node 0's side: edges 0,1 and 2,3, else 3,0 and 1,2).  Cells inside a body or with a
// non-finite value give none.  Output order: cell id j nx + i, then as above; three
// passes (count per block, scan of the block counts, write) keep that order.
namespace {

constexpr int CT_CELLS = 4;                  // consecutive cells per thread
constexpr int CT_CHUNK = BLOCK * CT_CELLS;   // cells per block

struct ContourArgs {
  int nx, ny;
  double x0, y0, hx, hy;
  const double* disp;  // component-major, (nx+1)(ny+1) each
  const int8_t* body;
  const double* f;
  double level;
  double* seg;         // (x0, y0, x1, y1) per segment
  long long cap;
  long long* boff;     // per block: segment count, then exclusive offset
  long long* total;
};

// Segments of cell cid (0, 1 or 2); their end points into out[0..8) when out != null.
__device__ int cell_contour(const ContourArgs& a, long long cid, double* out) {
  const int i = (int)(cid % a.nx), j = (int)(cid / a.nx);
  const long long nn = (long long)(a.nx + 1) * (a.ny + 1);
  const long long n0 = (long long)j * (a.nx + 1) + i;
  const long long nd[4] = {n0, n0 + 1, n0 + a.nx + 2, n0 + a.nx + 1};
  const int b0 = a.body[nd[0]];
  if (b0 >= 0 && a.body[nd[1]] == b0 && a.body[nd[2]] == b0 && a.body[nd[3]] == b0) return 0;
  double v[4];
  bool up[4];
  for (int k = 0; k < 4; ++k) {
    v[k] = a.f[nd[k]];
    if (!isfinite(v[k])) return 0;
    up[k] = v[k] >= a.level;
  }
  int ncross = 0;
  for (int e = 0; e < 4; ++e) ncross += up[e] != up[(e + 1) & 3];
  if (ncross == 0) return 0;
  const int nseg = ncross == 4 ? 2 : 1;
  if (!out) return nseg;
  const int oi[4] = {0, 1, 1, 0}, oj[4] = {0, 0, 1, 1};
  double cx[4], cy[4];
  for (int e = 0; e < 4; ++e) {
    const int p = e, q = (e + 1) & 3;
    if (up[p] == up[q]) continue;
    const double t = (a.level - v[p]) / (v[q] - v[p]);
    const double xp = (a.x0 + (double)(i + oi[p]) * a.hx) + a.disp[nd[p]];
    const double yp = (a.y0 + (double)(j + oj[p]) * a.hy) + a.disp[nd[p] + nn];
    const double xq = (a.x0 + (double)(i + oi[q]) * a.hx) + a.disp[nd[q]];
    const double yq = (a.y0 + (double)(j + oj[q]) * a.hy) + a.disp[nd[q] + nn];
    cx[e] = xp + t * (xq - xp);
    cy[e] = yp + t * (yq - yp);
  }
  if (nseg == 1) {
    int e0 = -1, e1 = -1;
    for (int e = 0; e < 4; ++e)
      if (up[e] != up[(e + 1) & 3]) {
        if (e0 < 0)
          e0 = e;
        else
          e1 = e;
      }
    out[0] = cx[e0];
    out[1] = cy[e0];
    out[2] = cx[e1];
    out[3] = cy[e1];
    return 1;
  }
  const bool centre_up = 0.25 * ((v[0] + v[1]) + (v[2] + v[3])) >= a.level;
  const int pr[4] = {0, 1, 2, 3}, ps[4] = {3, 0, 1, 2};
  const int* e = centre_up == up[0] ? pr : ps;
  for (int s = 0; s < 2; ++s) {
    out[4 * s] = cx[e[2 * s]];
    out[4 * s + 1] = cy[e[2 * s]];
    out[4 * s + 2] = cx[e[2 * s + 1]];
    out[4 * s + 3] = cy[e[2 * s + 1]];
  }
  return 2;
}

// Exclusive scan over the block of one long long per thread; returns the thread's
// offset and sets *sum to the block total.
__device__ long long block_exscan(long long v, long long* s_scan, long long* sum) {
  const int tid = threadIdx.x;
  s_scan[tid] = v;
  __syncthreads();
  for (int off = 1; off < BLOCK; off <<= 1) {
    const long long u = tid >= off ? s_scan[tid - off] : 0;
    __syncthreads();
    s_scan[tid] += u;
    __syncthreads();
  }
  const long long incl = s_scan[tid];
  *sum = s_scan[BLOCK - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(BLOCK) k_contour_count(ContourArgs a) {
  __shared__ long long s_scan[BLOCK];
  const long long ncell = (long long)a.nx * a.ny;
  const long long c0 = (long long)blockIdx.x * CT_CHUNK + (long long)threadIdx.x * CT_CELLS;
  long long cnt = 0;
  for (int c = 0; c < CT_CELLS; ++c)
    if (c0 + c < ncell) cnt += cell_contour(a, c0 + c, nullptr);
  long long sum;
  (void)block_exscan(cnt, s_scan, &sum);
  if (threadIdx.x == 0) a.boff[blockIdx.x] = sum;
}

// One block: block counts -> exclusive offsets, and the total.
__global__ void __launch_bounds__(BLOCK) k_contour_scan(ContourArgs a, int nblk) {
  __shared__ long long s_scan[BLOCK];
  const int per = (nblk + BLOCK - 1) / BLOCK;
  const int b0 = threadIdx.x * per;
  long long loc = 0;
  for (int k = 0; k < per; ++k)
    if (b0 + k < nblk) loc += a.boff[b0 + k];
  long long sum;
  long long off = block_exscan(loc, s_scan, &sum);
  for (int k = 0; k < per; ++k)
    if (b0 + k < nblk) {
      const long long c = a.boff[b0 + k];
      a.boff[b0 + k] = off;
      off += c;
    }
  if (threadIdx.x == 0) *a.total = sum;
}

__global__ void __launch_bounds__(BLOCK) k_contour_write(ContourArgs a) {
  __shared__ long long s_scan[BLOCK];
  const long long ncell = (long long)a.nx * a.ny;
  const long long c0 = (long long)blockIdx.x * CT_CHUNK + (long long)threadIdx.x * CT_CELLS;
  long long cnt = 0;
  for (int c = 0; c < CT_CELLS; ++c)
    if (c0 + c < ncell) cnt += cell_contour(a, c0 + c, nullptr);
  long long sum;
  long long idx = a.boff[blockIdx.x] + block_exscan(cnt, s_scan, &sum);
  for (int c = 0; c < CT_CELLS; ++c) {
    if (c0 + c >= ncell) break;
    double out[8];
    const int k = cell_contour(a, c0 + c, out);
    for (int s = 0; s < k; ++s, ++idx)
      if (idx < a.cap)
        for (int q = 0; q < 4; ++q) a.seg[4 * idx + q] = out[4 * s + q];
  }
}

long long contour_blocks(const mfp_grid* g) {
  const long long ncell = (long long)g->nx * g->ny;
  return (ncell + CT_CHUNK - 1) / CT_CHUNK;
}

}  // namespace

extern "C" size_t mfp_contour_workspace_size(const mfp_grid* grid) {
  if (!grid || grid->nx < 2 || grid->ny < 2) return 0;
  return (size_t)(contour_blocks(grid) + 1) * sizeof(long long) + 256;
}

extern "C" int mfp_contour(const mfp_grid* grid, const double* disp, const int8_t* body,
                           const double* field, double level, double* seg, int64_t cap,
                           int64_t* n_seg_h, void* ws, size_t ws_bytes, void* stream_) {
  clear_error();
  MFP_TRY(check_grid(grid));
  if (!disp || !body || !field || !n_seg_h || !ws || cap < 0 || (cap > 0 && !seg)) {
    set_error("NULL argument or negative cap");
    return MFP_E_ARG;
  }
  if (!std::isfinite(level)) {
    set_error("level is not finite");
    return MFP_E_ARG;
  }
  const long long nblk = contour_blocks(grid);
  if ((long long)grid->nx * grid->ny >= (1ll << 40)) {
    set_error("grid too large");
    return MFP_E_ARG;
  }
  const size_t need = mfp_contour_workspace_size(grid);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu", ws_bytes, need);
    return MFP_E_WORKSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream_);
  ContourArgs a{};
  a.nx = grid->nx;
  a.ny = grid->ny;
  a.x0 = grid->x0;
  a.y0 = grid->y0;
  a.hx = grid_hx(*grid);
  a.hy = grid_hy(*grid);
  a.disp = disp;
  a.body = body;
  a.f = field;
  a.level = level;
  a.seg = seg;
  a.cap = cap;
  a.boff = static_cast<long long*>(ws);
  a.total = a.boff + nblk;
  k_contour_count<<<(unsigned)nblk, BLOCK, 0, st>>>(a);
  k_contour_scan<<<1, BLOCK, 0, st>>>(a, (int)nblk);
  k_contour_write<<<(unsigned)nblk, BLOCK, 0, st>>>(a);
  MFP_TRY_HIP(hipGetLastError());
  long long total = 0;
  MFP_TRY_HIP(hipMemcpyAsync(&total, a.total, sizeof(long long), hipMemcpyDeviceToHost, st));
  MFP_TRY_HIP(hipStreamSynchronize(st));
  *n_seg_h = total;
  return MFP_OK;
}
