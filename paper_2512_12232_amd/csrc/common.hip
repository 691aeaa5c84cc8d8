// Host-side helpers of libmfpsi.so: thread-local error text, argument and geometry
// checks, node boxes around circles.
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "mfp_internal.h"

namespace mfp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int check_grid(const mfp_grid* g) {
  if (!g) {
    set_error("grid is NULL");
    return MFP_E_ARG;
  }
  if (g->nx < 2 || g->ny < 2) {
    set_error("grid needs at least 2x2 cells (got %d x %d)", g->nx, g->ny);
    return MFP_E_GEOMETRY;
  }
  if (!(g->x1 > g->x0) || !(g->y1 > g->y0)) {
    set_error("empty domain");
    return MFP_E_ARG;
  }
  // padded layout indices must fit comfortably in 32-bit tile arithmetic
  if ((long long)(g->nx + 1) * (g->ny + 1) > (1LL << 31) - (1LL << 24)) {
    set_error("grid too large");
    return MFP_E_ARG;
  }
  return MFP_OK;
}

// Same comparisons, in the same order, as the oracle's geometry check.
int check_geometry(const mfp_grid* g, const mfp_circle* c, int nb) {
  int s = check_grid(g);
  if (s) return s;
  if (nb < 0 || nb > MFP_MAX_BODIES) {
    set_error("nbody %d outside [0, %d]", nb, MFP_MAX_BODIES);
    return MFP_E_GEOMETRY;
  }
  if (nb > 0 && !c) {
    set_error("circles is NULL");
    return MFP_E_ARG;
  }
  const double hx = grid_hx(*g), hy = grid_hy(*g);
  const double h = hx > hy ? hx : hy;
  for (int b = 0; b < nb; ++b) {
    const double cx = c[b].cx, cy = c[b].cy, r = c[b].r;
    if (!(r >= 2.0 * h)) {
      set_error("circle %d: radius below two cells", b);
      return MFP_E_GEOMETRY;
    }
    if (!(cx - r >= g->x0 + hx && cx + r <= g->x1 - hx && cy - r >= g->y0 + hy &&
          cy + r <= g->y1 - hy)) {
      set_error("circle %d: within one cell of the outer boundary", b);
      return MFP_E_GEOMETRY;
    }
  }
  for (int a = 0; a < nb; ++a)
    for (int b = a + 1; b < nb; ++b) {
      const double dx = c[a].cx - c[b].cx, dy = c[a].cy - c[b].cy;
      const double rs = c[a].r + c[b].r;
      if (!(dx * dx + dy * dy > rs * rs)) {
        set_error("circles %d and %d overlap", a, b);
        return MFP_E_GEOMETRY;
      }
    }
  return MFP_OK;
}

Box circle_box(const mfp_grid& g, const mfp_circle& c, int pad, int ilo, int ihi, int jlo,
               int jhi) {
  const double hx = grid_hx(g), hy = grid_hy(g);
  Box b;
  b.i0 = (int)std::floor((c.cx - c.r - g.x0) / hx) - 1 - pad;
  b.i1 = (int)std::ceil((c.cx + c.r - g.x0) / hx) + 1 + pad;
  b.j0 = (int)std::floor((c.cy - c.r - g.y0) / hy) - 1 - pad;
  b.j1 = (int)std::ceil((c.cy + c.r - g.y0) / hy) + 1 + pad;
  b.i0 = b.i0 < ilo ? ilo : b.i0;
  b.j0 = b.j0 < jlo ? jlo : b.j0;
  b.i1 = b.i1 > ihi ? ihi : b.i1;
  b.j1 = b.j1 > jhi ? jhi : b.j1;
  return b;
}

}  // namespace mfp

extern "C" const char* mfp_last_error(void) { return mfp::g_err; }

extern "C" int mfp_check_geometry(const mfp_grid* grid, const mfp_circle* circles_h,
                                  int32_t nbody) {
  mfp::clear_error();
  return mfp::check_geometry(grid, circles_h, nbody);
}
