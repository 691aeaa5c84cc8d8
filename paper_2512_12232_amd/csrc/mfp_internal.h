// Internal definitions shared by the HIP sources of libmfpsi.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mfpsi.h"

namespace mfp {

// ---- errors ---------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

#define MFP_TRY_HIP(call)                                                        \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::mfp::set_error("%s failed: %s", #call, hipGetErrorString(e_));          \
      return MFP_E_HIP;                                                          \
    }                                                                            \
  } while (0)

#define MFP_TRY(expr)            \
  do {                           \
    int s_ = (expr);             \
    if (s_ < 0) return s_;       \
  } while (0)

// ---- geometry helpers (host) ------------------------------------------------------
int check_grid(const mfp_grid* g);
int check_geometry(const mfp_grid* g, const mfp_circle* c, int nb);
inline double grid_hx(const mfp_grid& g) { return (g.x1 - g.x0) / g.nx; }
inline double grid_hy(const mfp_grid& g) { return (g.y1 - g.y0) / g.ny; }

// Inclusive node-index box covering circle b, expanded by `pad` nodes and clipped to
// [lo, hi] in each direction.
struct Box {
  int i0, i1, j0, j1;
  bool empty() const { return i1 < i0 || j1 < j0; }
  long long count() const { return empty() ? 0 : (long long)(i1 - i0 + 1) * (j1 - j0 + 1); }
};
Box circle_box(const mfp_grid& g, const mfp_circle& c, int pad, int ilo, int ihi, int jlo,
               int jhi);

// ---- constrained solve with caller-given element entries (solve.hip) ---------------
// The single-system solve (as mfp_psi_solve, FP64, FP32 or FP32 + FP64 refinement) on
// an operator given cell by cell: cellcoef holds, entry-major, the six off-diagonal
// entries (k01, k02, k03, k12, k13, k23) of each cell's 4 x 4 matrix in the corner
// order (i, j), (i+1, j), (i+1, j+1), (i, j+1), rows summing to zero.  Nodes with
// body[n] = b >= 0 are tied to psi_b; psi receives the background-node values (tied
// nodes psi_b).  disp only marks the cells that are not plain rectangles.
size_t psi_solve_cells_workspace(const mfp_grid* grid, int nbody, const mfp_solver_opts* opts);
int psi_solve_cells(const mfp_grid* grid, const mfp_circle* circles_h, int nbody,
                    const double* disp, const int8_t* body, const double* cellcoef,
                    const mfp_flow* flow, const mfp_solver_opts* opts, int pair_lo,
                    int pair_hi, double* psi, double* psi_b_h, double* Q_h, double* copfi_h,
                    mfp_stats* stats_h, void* ws, size_t ws_bytes, hipStream_t st);
// The same with Kutta constraints (as mfp_psi_solve_kutta: kutta_xy_h holds (x, y) or
// (NaN, NaN) per body).
size_t psi_solve_cells_kutta_workspace(const mfp_grid* grid, int nbody, int nkutta,
                                       const mfp_solver_opts* opts);
int psi_solve_cells_kutta(const mfp_grid* grid, const mfp_circle* circles_h, int nbody,
                          const double* disp, const int8_t* body, const double* cellcoef,
                          const mfp_flow* flow, const mfp_solver_opts* opts,
                          const double* kutta_xy_h, int pair_lo, int pair_hi, double* psi,
                          double* psi_b_h, double* Q_h, double* copfi_h, int64_t* kutta_node_h,
                          mfp_stats* stats_h, void* ws, size_t ws_bytes, hipStream_t st);

// ---- workspace bump allocator ----------------------------------------------------
struct Bump {
  char* base;     // may be nullptr when only measuring
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

// ---- padded node layout used by the solver ----------------------------------------
// Node columns are grouped in strips of SW = 62; strip m occupies the 64-column,
// 512-byte-aligned block [64 m, 64 m + 63] of every padded row, its nodes at columns
// 64 m + 1 .. 64 m + 62; columns 64 m and 64 m + 63 are padding (tag TAG_HALO, zero
// in every vector).  Node (i, j) lives at (j+1) P + 64 (i / 62) + 1 + i % 62, with one
// halo row below and at least one above the domain.  The element apply works on
// "tasks": one wavefront per strip and chunk of HC node rows; lane l of strip m sits
// at column 64 m + l, lanes 1..62 own their node, lanes 0 and 63 read the nodes just
// left and right of the strip (at 64 m - 2 and 64 m + 65, see halo_shift) and store
// zeros into the padding, so that every row store is one whole aligned 512-byte line
// set.
constexpr int SW = 62;        // owned node columns per strip
constexpr int BLOCK = 256;    // 4 wavefronts, i.e. 4 tasks per block and step
constexpr int WAVES = BLOCK / 64;

struct Layout {
  int nx, ny;       // cells
  int hc;           // owned node rows per task (4 or 8)
  int nstrip;       // strips of SW owned columns
  int nchunk;       // chunks of hc owned rows
  int P;            // pitch (nodes per padded row), multiple of 64
  int rows;         // padded rows
  long long n;      // P * rows
  __host__ __device__ int ntasks() const { return nstrip * nchunk; }
};

// Tasks of 4 owned rows by default: consecutive tasks of a wavefront's segment share
// their halo rows in registers, so taller tasks save little traffic and cost
// registers (occupancy); hc_force = 8 selects 8-row tasks (FP32 solves of large
// grids).
inline Layout make_layout(int nx, int ny, int hc_force = 0) {
  Layout L;
  L.nx = nx;
  L.ny = ny;
  L.nstrip = (nx + 1 + SW - 1) / SW;
  L.hc = (hc_force == 8 || hc_force == 5) ? hc_force : 4;
  L.nchunk = (ny + 1 + L.hc - 1) / L.hc;
  L.P = 64 * L.nstrip;
  L.rows = L.hc * L.nchunk + 2;
  L.n = (long long)L.P * L.rows;
  return L;
}

// Padded index of node (i, j).
__host__ __device__ inline long long node_index(const Layout& L, int i, int j) {
  return (long long)(j + 1) * L.P + 64 * (i / SW) + 1 + (i % SW);
}

// Node column held at padded column col, or -1 for a padding column.
__host__ __device__ inline int column_node(int col) {
  const int l = col & 63;
  return (l == 0 || l == 63) ? -1 : (col >> 6) * SW + l - 1;
}

// Column shift from lane's own column to the column it reads: lanes 0 and 63 read
// the neighbouring strips' edge nodes (none beyond the first and last strip: there
// they read their own padding, a halo node).
__host__ __device__ inline int halo_shift(int lane, int m, int nstrip) {
  if (lane == 0) return m > 0 ? -2 : 0;
  if (lane == 63) return m + 1 < nstrip ? 2 : 0;
  return 0;
}

// Internal node tags.  For the stream function the nodes of body b carry
// TAG_BODY0 + b and stand for the one unknown psi_b.  For the velocity potential they
// carry -1 - b: unknowns of their own (no body constraint) whose tag still names the
// body, so that cells inside a body stay inactive.  Hence tag <= TAG_FREE: a node that
// is its own unknown; (uint8_t)tag >= TAG_BODY0: a body node of either kind.
enum : int8_t { TAG_FREE = 0, TAG_DIR = 1, TAG_HALO = 2, TAG_BODY0 = 3 };
__host__ __device__ inline int8_t tag_potential_body(int b) { return (int8_t)(-1 - b); }
__host__ __device__ inline bool tag_own(int8_t g) { return g <= TAG_FREE; }
__host__ __device__ inline bool tag_body(int8_t g) { return (uint8_t)g >= (uint8_t)TAG_BODY0; }

// Device-resident solver scalars.  Quantities that a kernel reads for iteration k
// while its block 0 writes the value for the next iteration are double-buffered by
// iteration parity, so no kernel reads a slot that the same launch writes.
struct DevState {
  double rr[2];                          // r.r of iterate k in slot k&1
  double rb_rr[2];                       // body part of r.r of iterate k in slot k&1
  double pb[2][MFP_MAX_BODIES];          // body directions p_b of iteration k, slot k&1
  double xb[2][MFP_MAX_BODIES];          // body unknowns of iterate k, slot k&1
  double rb[2][MFP_MAX_BODIES];          // body residuals of iterate k, slot k&1
  double qb[MFP_MAX_BODIES];             // body sums of the last plain apply
  double bb[MFP_MAX_BODIES];             // extra right-hand side of the body rows (adjoint)
  double rr0, rr_stop, rr_final, rr_true;
  double alpha, beta, pq;
  double rr_prev;                        // one-kernel CG: |r|^2 before a restart (0: fresh)
  double alpha_hist[2];                  // one-kernel CG: alpha_{k-1} computed by launch k, slot k&1
  long long jbase;                       // batched one-kernel CG: first launch of the replay
  long long k0;                          // batched one-kernel CG: start launch of the run
  double stop_rel;                       // one-kernel CG: threshold / start |r|^2 (0: use rr_stop)
  double copfi, Q;
  long long iters;                       // index of the final iterate once done != 0
  long long kmax;
  long long outer_count;                 // batched mixed solves: FP64 refinements so far
  int done;                              // 0 running, 1 converged, 2 breakdown, 3 kmax
  int pad_;
};

}  // namespace mfp
