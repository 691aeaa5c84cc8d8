// Matrix-free Q1 element operator on the padded node layout.
//
// The paper's Algorithm 1 (appendix) loops over elements, multiplies each element
// matrix with the element extract of the global vector and accumulates the element
// results into the global vector; its element matrices are K_e = int (grad N)^T
// (grad N) dOmega (section "Weak formulation").  Here the element matrix is never
// stored: each workgroup owns a 64 x 8 tile of nodes, stages the tile plus a
// one-node halo in LDS, evaluates K_e(X_e) p_e for every cell touching the tile with
// the 2x2 Gauss rule from the node displacements, parks the four results of each
// cell in LDS and lets every owned node gather the contributions of its four cells.
// Each output is written exactly once, so no atomics and no colouring of the global
// scatter are needed.  Tiles whose footprint holds only free, undisplaced nodes take
// the assembled constant 9-point stencil of the rectangular cell instead (same
// operator, a few ulp apart).
#pragma once

#include "mfp_internal.h"

namespace mfp {

// Sum over a 256-thread block; every thread receives the total.  Fixed reduction
// order, so results are reproducible run to run.
__device__ __forceinline__ double block_sum(double v, double* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) s_red[tid >> 6] = v;
  __syncthreads();
  const double t = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  return t;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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

template <typename T>
struct ApplyArgs {
  int P, ntx, ntiles, tpb;       // pitch, tiles per row, tile count, tiles per block
  const int8_t* tag;
  const T* dx;                   // displacement / hx
  const T* dy;
  const uint8_t* tplain;         // 1: constant-stencil tile
  const unsigned long long* tbody;  // bodies among the tile's own nodes
  const int* tslot;              // body-partial slot of the tile or -1
  const T* src;                  // plain apply: p; fused: previous direction
  const T* r;                    // fused: residual
  T* pnew;                       // fused: new direction (written at own nodes)
  T* q;                          // K p at free nodes (all in-domain nodes if write_all)
  double* part;                  // per-block partial of p.q over free nodes
  double* bpart;                 // per-slot, per-body partial sums of K p
  const double* part2;           // fused: per-block partials of r.r from the update
  int G2;                        // fused: number of those partials
  long long k;                   // fused: iteration index
  DevState* st;
  int nb;
  int write_all;
  T cC, cE, cN, cD;              // constant stencil (centre, east/west, north/south, diag)
  T ry;                          // hy / hx
};

// FUSED = false: q = K src.
// FUSED = true: one CG iteration's first half.  Every block reduces the previous
// update's r.r partials itself (identical order in every block, so identical
// results), forms beta = r_k.r_k / r_{k-1}.r_{k-1} and the body directions, stops
// the solve when the tolerance, kmax or a non-finite value is reached, and then forms
// p = r + beta p_old (body nodes p_b, Dirichlet nodes 0) before applying K.
// There is no grid-wide synchronisation inside the kernel: partial sums go to
// per-block slots that the next kernel reduces.
template <typename T, bool FUSED>
__global__ void __launch_bounds__(BLOCK) k_apply(ApplyArgs<T> a) {
  __shared__ T s_p[FH][FW];
  __shared__ T s_dx[FH][FW];
  __shared__ T s_dy[FH][FW];
  __shared__ int8_t s_tag[FH][FW];
  __shared__ T s_c[4][CH][CW];
  __shared__ double s_red[BLOCK / 64];
  __shared__ double s_pb[MFP_MAX_BODIES];

  const int tid = threadIdx.x;
  if (FUSED && a.st->done) return;
  const int G = gridDim.x;
  // consecutive virtual blocks share an XCD (work-groups are dealt round-robin to 8 XCDs)
  const int vb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int t0 = vb * a.tpb;
  const int t1 = min(t0 + a.tpb, a.ntiles);
  const long long P = a.P;

  // Footprint values of the next tile are held in registers (NE per thread) so that
  // its loads are in flight while the current tile is computed.
  constexpr int NE = (FH * FW + BLOCK - 1) / BLOCK;
  T ra[NE], rb[NE], rdx[NE], rdy[NE];
  int8_t rtag[NE];
  auto issue = [&](int t, bool plain) {
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const long long base = (long long)(ty * TY) * P + tx * TX;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = tid + k * BLOCK;
      if (e < FH * FW) {
        const int fr = e / FW, fc = e - fr * FW;
        const long long gi = base + fr * P + fc;
        rb[k] = a.src[gi];
        if (FUSED) ra[k] = a.r[gi];
        if (!plain) {
          rtag[k] = a.tag[gi];
          rdx[k] = a.dx[gi];
          rdy[k] = a.dy[gi];
        }
      }
    }
  };
  bool plain_next = t0 < t1 ? a.tplain[t0] != 0 : true;
  if (t0 < t1) issue(t0, plain_next);

  T beta = (T)0;
  if (FUSED) {
    DevState* st = a.st;
    const int cur = (int)(a.k & 1), prv = cur ^ 1;
    double s = 0.0;
    for (int i = tid; i < a.G2; i += BLOCK) s += a.part2[i];
    const double rrk = block_sum(s, s_red) + st->rb_rr[cur];
    const double beta_d = rrk / st->rr[prv];
    int code = 0;
    if (!isfinite(rrk))
      code = 2;
    else if (rrk <= st->rr_stop)
      code = 1;
    else if (a.k >= st->kmax)
      code = 3;
    if (code) {
      if (blockIdx.x == 0 && tid == 0) {
        st->done = code;
        st->iters = a.k;
        st->rr_final = rrk;
      }
      return;
    }
    if (tid < a.nb) {
      const double v = st->rb[cur][tid] + beta_d * st->pb[prv][tid];
      s_pb[tid] = v;
      if (blockIdx.x == 0) st->pb[cur][tid] = v;
    }
    if (blockIdx.x == 0 && tid == 0) {
      st->rr[cur] = rrk;
      st->beta = beta_d;
    }
    beta = (T)beta_d;
    __syncthreads();
  }

  double pq = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const long long base = (long long)(ty * TY) * P + tx * TX;
    const bool plain = plain_next;
    // registers -> LDS (forming the new direction on the way in the fused form)
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = tid + k * BLOCK;
      if (e < FH * FW) {
        const int fr = e / FW, fc = e - fr * FW;
        T v;
        if (FUSED) {
          if (plain) {
            v = ra[k] + beta * rb[k];
          } else {
            const int8_t tg = rtag[k];
            v = tg == TAG_FREE ? ra[k] + beta * rb[k]
                               : (tg >= TAG_BODY0 ? (T)s_pb[tg - TAG_BODY0] : (T)0);
          }
          if (fr >= 1 && fr <= TY && fc >= 1 && fc <= TX) a.pnew[base + fr * P + fc] = v;
        } else {
          v = rb[k];
        }
        s_p[fr][fc] = v;
        if (!plain) {
          s_tag[fr][fc] = rtag[k];
          s_dx[fr][fc] = rdx[k];
          s_dy[fr][fc] = rdy[k];
        }
      }
    }
    if (t + 1 < t1) {
      plain_next = a.tplain[t + 1] != 0;
      issue(t + 1, plain_next);
    }
    __syncthreads();
    if (plain) {
#pragma unroll
      for (int k = 0; k < (TX * TY) / BLOCK; ++k) {
        const int o = tid + k * BLOCK;
        const int rr = 1 + o / TX, cc = 1 + (o % TX);
        const T c = s_p[rr][cc];
        const T v = a.cC * c + a.cE * (s_p[rr][cc - 1] + s_p[rr][cc + 1]) +
                    a.cN * (s_p[rr - 1][cc] + s_p[rr + 1][cc]) +
                    a.cD * ((s_p[rr - 1][cc - 1] + s_p[rr - 1][cc + 1]) +
                            (s_p[rr + 1][cc - 1] + s_p[rr + 1][cc + 1]));
        a.q[base + rr * P + cc] = v;
        pq += (double)c * (double)v;
      }
    } else {
      for (int c = tid; c < CH * CW; c += BLOCK) {
        const int cr = c / CW, cc = c - cr * CW;
        const int8_t g0 = s_tag[cr][cc], g1 = s_tag[cr][cc + 1], g2 = s_tag[cr + 1][cc + 1],
                     g3 = s_tag[cr + 1][cc];
        const bool halo = (g0 == TAG_HALO) | (g1 == TAG_HALO) | (g2 == TAG_HALO) | (g3 == TAG_HALO);
        const bool inside = (g0 >= TAG_BODY0) & (g1 == g0) & (g2 == g0) & (g3 == g0);
        T y0 = 0, y1 = 0, y2 = 0, y3 = 0;
        if (!halo && !inside) {
          cell_apply<T>(a.ry, s_dx[cr][cc], s_dx[cr][cc + 1], s_dx[cr + 1][cc + 1],
                        s_dx[cr + 1][cc], s_dy[cr][cc], s_dy[cr][cc + 1],
                        s_dy[cr + 1][cc + 1], s_dy[cr + 1][cc], s_p[cr][cc],
                        s_p[cr][cc + 1], s_p[cr + 1][cc + 1], s_p[cr + 1][cc], y0, y1, y2,
                        y3);
        }
        s_c[0][cr][cc] = y0;
        s_c[1][cr][cc] = y1;
        s_c[2][cr][cc] = y2;
        s_c[3][cr][cc] = y3;
      }
      __syncthreads();
      T sums[(TX * TY) / BLOCK];
      int8_t tags[(TX * TY) / BLOCK];
#pragma unroll
      for (int k = 0; k < (TX * TY) / BLOCK; ++k) {
        const int o = tid + k * BLOCK;
        const int rr = 1 + o / TX, cc = 1 + (o % TX);
        const T sum = (s_c[2][rr - 1][cc - 1] + s_c[3][rr - 1][cc]) +
                      (s_c[1][rr][cc - 1] + s_c[0][rr][cc]);
        const int8_t tg = s_tag[rr][cc];
        const bool keep = (tg == TAG_FREE) || (a.write_all && tg != TAG_HALO);
        a.q[base + rr * P + cc] = keep ? sum : (T)0;
        if (tg == TAG_FREE) pq += (double)s_p[rr][cc] * (double)sum;
        sums[k] = sum;
        tags[k] = tg;
      }
      const unsigned long long bm = a.tbody[t];
      if (bm) {
        const int slot = a.tslot[t];
        for (int b = 0; b < a.nb; ++b) {
          if (bm & (1ull << b)) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < (TX * TY) / BLOCK; ++k)
              if (tags[k] == TAG_BODY0 + b) v += (double)sums[k];
            v = block_sum(v, s_red);
            if (tid == 0) a.bpart[(long long)slot * a.nb + b] = v;
          } else if (tid == 0) {
            a.bpart[(long long)slot * a.nb + b] = 0.0;
          }
        }
      }
    }
    __syncthreads();
  }
  const double bsum = block_sum(pq, s_red);
  if (tid == 0) a.part[blockIdx.x] = bsum;
}

// Per-body sums of the slot partials, into s_qb[0 .. nb); wave w handles bodies
// w, w+4, ...  Fixed order.
__device__ __forceinline__ void body_sums(const double* __restrict__ bpart, int nslots, int nb,
                                          double* s_qb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int b = w; b < nb; b += BLOCK / 64) {
    double v = 0.0;
    for (int sl = lane; sl < nslots; sl += 64) v += bpart[(long long)sl * nb + b];
    v = wave_sum(v);
    if (lane == 0) s_qb[b] = v;
  }
  __syncthreads();
}

}  // namespace mfp
