// gfx950 kernels of the multigrid elasticity solver.  One thread per node,
// 64 x 4 thread blocks (one wavefront per x-row of a tile), x fastest so
// every load of a field component is a coalesced row of 64 nodes.
#pragma once
#include <algorithm>
#include <type_traits>
#include "emg_device.hpp"

namespace emg {

enum { MODE_APPLY = 0, MODE_RESID = 1, MODE_JACOBI = 2 };

constexpr int BX = 64, BY = 4;

// Tile shapes (x extent x y extent of one plane) of the tile kernel and of
// the restriction and interpolation launches, chosen per level by the
// autotuner; 64 x 4 unless tuned (batched launches always use 64 x 4).
enum { TS_64x4 = 0, TS_64x2 = 1, TS_128x2 = 2, TS_32x8 = 3, TS_COUNT = 4 };
__host__ __device__ constexpr int ts_x(int s) { return s == TS_128x2 ? 128 : (s == TS_32x8 ? 32 : 64); }
__host__ __device__ constexpr int ts_y(int s) { return s == TS_64x4 ? 4 : (s == TS_32x8 ? 8 : 2); }

__device__ __forceinline__ bool skip(const Ctl *ctl) { return ctl != nullptr && ctl->done != 0; }

__device__ __forceinline__ long long block_linear() {
  return ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

// XCD-aware tile order.  Workgroups are dealt to the 8 XCDs round-robin in
// dispatch order, and each XCD has its own L2.  Renumber them so that XCD x
// walks one contiguous run of tiles (x fastest, then y, then z): its tiles'
// y- and z-neighbours then sit in the same L2 instead of being fetched again
// from HBM by another XCD.  Returns the tile coordinates of this block.
constexpr int kXCD = 8;
__device__ __forceinline__ unsigned tile_of(int &tx, int &ty, int &tz) {
  const unsigned B = gridDim.x * gridDim.y * gridDim.z;
  const unsigned b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const unsigned q = B / kXCD, r = B % kXCD;
  const unsigned x = b % kXCD, i = b / kXCD;
  const unsigned L = x * q + (x < r ? x : r) + i;
  tx = L % gridDim.x;
  ty = (L / gridDim.x) % gridDim.y;
  tz = L / (gridDim.x * gridDim.y);
  return L;
}

// Tile of this block from a list of active tiles (refined AMR levels: the
// 64 x 4 tiles of a plane that hold valid nodes or their ghosts), or the
// XCD-aware order over the whole grid when act is null.
__device__ __forceinline__ void tile_in(const int *__restrict__ act, int m0, int m1, int &tx, int &ty, int &tz) {
  if (!act) {
    tile_of(tx, ty, tz);
    return;
  }
  const int gx = (m0 + BX - 1) / BX, gy = (m1 + BY - 1) / BY;
  const int L = act[blockIdx.x];
  tx = L % gx;
  ty = (L / gx) % gy;
  tz = L / (gx * gy);
}

// Work decomposition of a stencil pass over one level.  The interior box
// holds the nodes whose rows are interior rows with in-range or periodically
// wrapped neighbours: per axis the full range if periodic, else 1..m-2.  The
// shell is the rest (boundary rows).  Blocks of 256 shell nodes come first,
// then tiles of 64 x 4 nodes of one plane over the box, so the slower shell
// blocks overlap the tiles instead of forming a tail.  Interior tiles take a
// path with no row classification.  Block index = norm-partial index.
struct Split {
  int lo[3], hi[3];     // interior box per axis (inclusive)
  int ntx, nty, ntz;    // interior tiles per axis (all 0 if the box is empty)
  long long inner;      // interior tiles
  long long shell;      // shell nodes
  long long sblocks;    // ceil(shell / 256)
  long long blocks;     // sblocks + inner
};

template <int TX = BX, int TY = BY>
__host__ __device__ inline Split split_tiles(const Geom &g) {
  Split s;
  long long box = 1;
  bool empty = false;
  for (int a = 0; a < 3; a++) {
    if (a >= g.dim) {
      s.lo[a] = 0;
      s.hi[a] = 0;
    } else if (g.per[a]) {
      s.lo[a] = 0;
      s.hi[a] = g.m[a] - 1;
    } else {
      s.lo[a] = 1;
      s.hi[a] = g.m[a] - 2;
    }
    const int b = s.hi[a] - s.lo[a] + 1;
    if (b <= 0) empty = true;
    box *= b > 0 ? b : 0;
  }
  if (!empty) {
    s.ntx = (s.hi[0] - s.lo[0] + TX) / TX;
    s.nty = (s.hi[1] - s.lo[1] + TY) / TY;
    s.ntz = s.hi[2] - s.lo[2] + 1;
    s.inner = (long long)s.ntx * s.nty * s.ntz;
    s.shell = g.N - box;
  } else {
    s.ntx = s.nty = s.ntz = 0;
    s.inner = 0;
    s.shell = g.N;
  }
  s.sblocks = (s.shell + TX * TY - 1) / (TX * TY);
  s.blocks = s.sblocks + s.inner;
  return s;
}
__host__ __device__ inline Split split_of(const Geom &g) { return split_tiles<BX, BY>(g); }
// host: the split of a tile shape chosen at run time
inline Split split_shape(const Geom &g, int shape) {
  switch (shape) {
    case TS_64x2: return split_tiles<64, 2>(g);
    case TS_128x2: return split_tiles<128, 2>(g);
    case TS_32x8: return split_tiles<32, 8>(g);
    default: return split_tiles<64, 4>(g);
  }
}

// Coordinates of shell node s: the planes below the box (z < lo), then for
// every box plane its ring (full rows outside the box, then the columns
// outside the box of the box rows), then the planes above the box.  With an
// empty box the shell is every node in storage order.
__device__ __forceinline__ void shell_node(const Geom &g, const Split &sp, long long s, int p[3]) {
  const int m0 = g.m[0], m1 = g.m[1];
  const long long plane = (long long)m0 * m1;
  if (sp.inner == 0) {
    p[0] = int(s % m0);
    p[1] = int((s / m0) % m1);
    p[2] = int(s / plane);
    return;
  }
  const int nzlo = sp.lo[2], nylo = sp.lo[1], nyhi = m1 - 1 - sp.hi[1], nxlo = sp.lo[0], nxhi = m0 - 1 - sp.hi[0];
  const int by = sp.hi[1] - sp.lo[1] + 1;
  if (s < nzlo * plane) {
    p[2] = int(s / plane);
    p[0] = int(s % m0);
    p[1] = int((s / m0) % m1);
    return;
  }
  s -= nzlo * plane;
  const long long ring = (long long)(nylo + nyhi) * m0 + (long long)by * (nxlo + nxhi);
  if (s < sp.ntz * ring) {
    p[2] = sp.lo[2] + int(s / ring);
    long long t = s % ring;
    if (t < (long long)nylo * m0) {
      p[1] = 0;
      p[0] = int(t);
      return;
    }
    t -= (long long)nylo * m0;
    if (t < (long long)nyhi * m0) {
      p[1] = m1 - 1;
      p[0] = int(t);
      return;
    }
    t -= (long long)nyhi * m0;
    const int cpr = nxlo + nxhi;
    p[1] = sp.lo[1] + int(t / cpr);
    p[0] = int(t % cpr) < nxlo ? 0 : m0 - 1;
    return;
  }
  s -= sp.ntz * ring;
  p[2] = sp.hi[2] + 1 + int(s / plane);
  p[0] = int(s % m0);
  p[1] = int((s / m0) % m1);
}

// Operator application / residual / damped Jacobi sweep on one level.
//   APPLY : out = D_H u
//   RESID : out = f - D_H u                (norm partials if `partial`)
//   JACOBI: out = u + omega (f - D_H u)/diag, Dirichlet rows out = f
//           (norm partials of f - D_H u, i.e. of the input's residual, if `partial`)
// Norm partials sum squares over non-Dirichlet rows, one value per block.
template <int MODE, int D, typename R, typename TO>
__device__ __forceinline__ void finish_rows(long long N, long long n, int cls, const R acc[D], const R dg[D],
                                            const R *__restrict__ u, const R *__restrict__ f, TO *__restrict__ out,
                                            R omega, double &nrm) {
#pragma unroll
  for (int i = 0; i < D; i++) {
    const long long q = i * N + n;
    if constexpr (MODE == MODE_APPLY) {
      out[q] = TO(acc[i]);
    } else if constexpr (MODE == MODE_RESID) {
      const R r = f[q] - acc[i];
      out[q] = TO(r);
      if (cls != ROW_DIR) nrm += double(r) * double(r);
    } else {
      const R r = f[q] - acc[i];
      if (cls == ROW_DIR) {
        out[q] = TO(f[q]);
      } else {
        out[q] = TO(u[q] + omega * r / dg[i]);
        nrm += double(r) * double(r);
      }
    }
  }
}

// MASK (refined AMR levels): nodes of the interior box whose byte in vm is 0
// (not valid: ghosts and nodes outside every box of the level) take the
// Dirichlet row instead, as the outer ring of the level's array does.
template <int D, int K, typename R, int MODE, typename TO, bool MASK = false, int TX = BX, int TY = BY>
__device__ __forceinline__ void body_stencil(const Geom &g, const R *__restrict__ C, const R *__restrict__ u,
                                             const R *__restrict__ f, TO *__restrict__ out, R omega,
                                             double *__restrict__ pslot, long long t,
                                             const unsigned char *__restrict__ vm = nullptr,
                                             const int lx = threadIdx.x, const int ly = threadIdx.y) {
  static_assert(!MASK || MODE != MODE_APPLY, "masked passes are residuals and sweeps");
  const Split sp = split_tiles<TX, TY>(g);
  double nrm = 0.0;
  if (t >= sp.sblocks) {
    const long long it = t - sp.sblocks;
    const int tx = int(it % sp.ntx), ty = int((it / sp.ntx) % sp.nty), tz = int(it / ((long long)sp.ntx * sp.nty));
    const int x = sp.lo[0] + tx * TX + lx, y = sp.lo[1] + ty * TY + ly, z = sp.lo[2] + tz;
    if (x <= sp.hi[0] && y <= sp.hi[1]) {
      // 32-bit node indexing (level sizes are checked at creation: N < 2^31)
      const unsigned m0 = g.m[0], m01 = (unsigned)g.m[0] * g.m[1];
      const unsigned n = z * m01 + y * m0 + x;
      const int c[3] = {x, y, z};
      const unsigned st[3] = {1u, m0, m01};
      unsigned om[3], op[3];
#pragma unroll
      for (int a = 0; a < 3; a++) {   // periodic wrap on the box faces of periodic axes
        om[a] = a < D ? (c[a] == 0 ? (g.m[a] - 1) * st[a] : 0u - st[a]) : 0u;
        op[a] = a < D ? (c[a] == g.m[a] - 1 ? 0u - (g.m[a] - 1) * st[a] : st[a]) : 0u;
      }
      R i2h[3], ih2[3];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        i2h[a] = R(0.5 / g.h[a]);
        ih2[a] = R(1.0 / (g.h[a] * g.h[a]));
      }
      R acc[D], dg[D], uc[D], fc[D];
      interior_rows<D, K, R, PtrU<R>, unsigned>(C, g.SC, PtrU<R>{u, g.N}, n, om, op, i2h, ih2, acc, dg,
                                                MODE == MODE_APPLY ? nullptr : f, g.N, fc, uc);
      const bool valid = !MASK || vm[n] != 0;
#pragma unroll
      for (int i = 0; i < D; i++) {   // interior rows (unless masked out): never Dirichlet
        TO *__restrict__ oi = (TO *)((char *)(out + i * g.N) + n * (unsigned)sizeof(TO));
        if constexpr (MODE == MODE_APPLY) {
          *oi = TO(acc[i]);
        } else {
          const R r = fc[i] - acc[i];
          if (valid) {
            *oi = MODE == MODE_RESID ? TO(r) : TO(uc[i] + omega * r / dg[i]);
            nrm += double(r) * double(r);
          } else {
            *oi = MODE == MODE_RESID ? TO(fc[i] - uc[i]) : TO(fc[i]);
          }
        }
      }
    }
  } else {
    const long long s = t * (TX * TY) + lx + TX * ly;
    if (s < sp.shell) {
      int p[3];
      shell_node(g, sp, s, p);
      const long long n = ((long long)p[2] * g.m[1] + p[1]) * g.m[0] + p[0];
      const int cls = row_class(g, p);
      R acc[D], dg[D];
      rows_at<D, K, R>(g, C, PtrU<R>{u, g.N}, n, p, cls, acc, dg);
      finish_rows<MODE, D, R, TO>(g.N, n, cls, acc, dg, u, f, out, omega, nrm);
    }
  }
  if (pslot) {
    if constexpr (TX * TY == 256) block_sum_256(nrm, pslot);
    else block_sum_128(nrm, pslot);
  }
}

// The tile kernel on a refined AMR level: rows of nodes that are not valid
// (vm[n] == 0) are Dirichlet rows.  Blocks: the shell blocks, then the
// interior tiles listed in act (those holding valid nodes or ghosts; the
// other nodes are never read).
template <int D, int K, typename R, int MODE, typename TO>
__global__ __launch_bounds__(256, 2) void k_stencil_mask(Geom g, const R *__restrict__ C, const R *__restrict__ u,
                                                      const R *__restrict__ f, TO *__restrict__ out, R omega,
                                                      const unsigned char *__restrict__ vm,
                                                      const int *__restrict__ act, long long sblocks,
                                                      const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  const long long b = blockIdx.x;
  const long long t = b < sblocks ? b : sblocks + act[b - sblocks];
  body_stencil<D, K, R, MODE, TO, true>(g, C, u, f, out, omega, nullptr, t, vm);
}

// One launch of split_of(g).blocks workgroups (64 x 4 threads) in dispatch
// order (an XCD-contiguous order of the tiles measured 3-4 % slower); at
// least two wavefronts per SIMD (the FP64 anisotropic path would otherwise
// take just over the 256 registers of that occupancy).
template <int D, int K, typename R, int MODE, typename TO, int TX = BX, int TY = BY>
__global__ __launch_bounds__(TX * TY, 2) void k_stencil(Geom g, const R *__restrict__ C,
                                                                    const R *__restrict__ u, const R *__restrict__ f,
                                                                    TO *__restrict__ out, R omega,
                                                                    double *__restrict__ partial,
                                                                    const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  const long long t = blockIdx.x;
  body_stencil<D, K, R, MODE, TO, false, TX, TY>(g, C, u, f, out, omega, partial ? partial + t : nullptr, t);
}

// ---- z-marching interior pass (3D, anisotropic moduli) ----
// A workgroup of 64 x 4 threads walks one column of interior tiles (the
// tiles of body_stencil) through a run of planes.  The moduli of the current
// plane and the displacement of three consecutive planes sit in LDS with a
// one-node halo in x and y, so every neighbour value of the 19-point stencil
// and every x/y neighbour modulus row comes from LDS: per node the pass
// issues about 40 global loads (each value once, plus the halo) instead of
// about 170, which on this GPU are bound by the vector-memory address rate,
// not by HBM.  The -z modulus rows are the previous plane's centre moduli,
// kept in registers; the +z rows of plane z are applied one step later, when
// plane z+1's moduli are the LDS centre, so the next plane's loads are only
// consumed by the LDS store at the end of a step and are issued in four
// groups spread over its compute phases.  Arithmetic, its order, and the
// norm partial of each 64 x 4 tile (its slot and summation order) are those
// of the interior tiles of body_stencil, bit for bit.
constexpr int ZM_HX = BX + 2, ZM_HY = BY + 2, ZM_HP = ZM_HX * ZM_HY, ZM_NH = ZM_HP - BX * BY;

// Chunks per column of a z-marching pass (workgroups = columns x chunks), or
// 0 if the level is better served by body_stencil (fewer than 8 planes per
// chunk).  target_wg workgroups are resident at once; the count minimises
// rounds x (planes per chunk + 7), the 7 standing for a chunk's priming and a
// round's ramp and tail (measured on 97^3, 129^3, 193^3 and 257^3 levels: a
// part-filled last round costs as much as a full one, and every chunk start
// re-reads two planes).  All columns share the chunk boundaries, so the
// workgroups of a round march level with one another.
__host__ inline int zm_chunks(const Geom &g, int target_wg) {
  if (g.dim != 3) return 0;
  const Split sp = split_of(g);
  if (sp.inner == 0) return 0;
  const long long cols = (long long)sp.ntx * sp.nty;
  int best = 0;
  long long best_cost = 0;
  for (int nzc = 1; nzc <= sp.ntz / 8; nzc++) {
    const long long rounds = (cols * nzc + target_wg - 1) / target_wg;
    const long long cost = rounds * ((sp.ntz + nzc - 1) / nzc + 7);
    if (best == 0 || cost < best_cost) {
      best = nzc;
      best_cost = cost;
    }
  }
  return best;
}

// xz (FP64 residual to FP32 only): also write the FP32 correction cycle's
// first sweep from zero, xz = omegaf r32 / diag32 (diag32 from the moduli
// rounded to FP32), the values k_jacobi_zero<float> would give.
template <typename R, int MODE, typename TO>
__device__ __forceinline__ void zm_column(const Geom &g, const Split &sp, const R *__restrict__ C, const R *__restrict__ u,
                                          const R *__restrict__ f, TO *__restrict__ out, R omega,
                                          double *__restrict__ partial, int nzc, unsigned w, R *__restrict__ sC,
                                          R *__restrict__ sU, float *__restrict__ xz = nullptr, float omegaf = 0.0f) {
  constexpr bool JZ = MODE == MODE_RESID && std::is_same<R, double>::value && std::is_same<TO, float>::value;
  constexpr int TX = BX, TY = BY, HX = ZM_HX, HY = ZM_HY, HP = ZM_HP, NH = ZM_NH, NC = 21, NV = 6;
  constexpr int HW = (NH + 63) / 64;   // wavefronts holding a halo position
  const int tx = threadIdx.x, ty = threadIdx.y, t = ty * TX + tx;
  const int wave = __builtin_amdgcn_readfirstlane(ty);
  const unsigned nwg = (unsigned)sp.ntx * sp.nty * nzc;
  // XCD x (workgroups x, x+8, ...) takes a contiguous run of columns, so the
  // halo rows shared by neighbouring columns are fetched into one L2
  const unsigned L = nwg % kXCD == 0 ? (w % kXCD) * (nwg / kXCD) + w / kXCD : w;
  const int chunk = L % nzc, col = L / nzc;
  const int cx = col % sp.ntx, cy = col / sp.ntx;
  const int x0 = sp.lo[0] + cx * TX, y0 = sp.lo[1] + cy * TY;
  const int nz = sp.hi[2] - sp.lo[2] + 1;
  const int zs = sp.lo[2] + (int)((long long)nz * chunk / nzc);
  const int ze = sp.lo[2] + (int)((long long)nz * (chunk + 1) / nzc);
  const int m0 = g.m[0], m1 = g.m[1], m2 = g.m[2];
  // coordinates of a tile or halo position: wrapped on periodic axes,
  // clamped otherwise (clamped positions only feed lanes outside the box)
  auto fix = [](int c, int m, int per) {
    if (per) {
      c %= m;
      return c < 0 ? c + m : c;
    }
    return c < 0 ? 0 : (c > m - 1 ? m - 1 : c);
  };
  const bool inbox = x0 + tx <= sp.hi[0] && y0 + ty <= sp.hi[1];
  const int p0 = (ty + 1) * HX + tx + 1;
  const unsigned r0 = (unsigned)fix(y0 + ty, m1, g.per[1]) * m0 + fix(x0 + tx, m0, g.per[0]);
  int p1 = p0;   // lanes of halo wavefronts without a halo position repeat their own node
  unsigned r1 = r0;
  if (t < NH) {
    int hx, hy;
    if (t < HX) {
      hy = 0;
      hx = t;
    } else if (t < 2 * HX) {
      hy = HY - 1;
      hx = t - HX;
    } else {
      const int q = t - 2 * HX;
      hy = 1 + q / 2;
      hx = (q & 1) ? HX - 1 : 0;
    }
    p1 = hy * HX + hx;
    r1 = (unsigned)fix(y0 + hy - 1, m1, g.per[1]) * m0 + fix(x0 + hx - 1, m0, g.per[0]);
  }
  const bool halo = wave < HW;
  // component bases in 64-bit arithmetic, node offsets in 32 bits (N < 2^29)
  const unsigned P = (unsigned)m0 * m1;
  const long long N = g.N, SC = g.SC;
  auto plane = [&](int z) {
    if (g.per[2]) z = z < 0 ? z + m2 : (z >= m2 ? z - m2 : z);
    return (unsigned)z * P;
  };
  R i2h[3], ih2[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    i2h[a] = R(0.5 / g.h[a]);
    ih2[a] = R(1.0 / (g.h[a] * g.h[a]));
  }
  // next plane's values in flight: moduli (own node, halo node), displacement, right-hand side
  R xc0[NC], xc1[NC], xu0[3], xu1[3], xf[3];
  auto issue = [&](int zc, int zu, int zf, int q) {
    const unsigned oc = plane(zc), ou = plane(zu);
    if (q == 0) {
#pragma unroll
      for (int c = 0; c < 11; c++) xc0[c] = ld(C + c * SC, oc + r0);
    } else if (q == 1) {
#pragma unroll
      for (int c = 11; c < NC; c++) xc0[c] = ld(C + c * SC, oc + r0);
    } else if (q == 2) {
      if (halo) {
#pragma unroll
        for (int c = 0; c < NC; c++) xc1[c] = ld(C + c * SC, oc + r1);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 3; k++) xu0[k] = ld(u + k * N, ou + r0);
      if (halo) {
#pragma unroll
        for (int k = 0; k < 3; k++) xu1[k] = ld(u + k * N, ou + r1);
      }
      if constexpr (MODE != MODE_APPLY) {
#pragma unroll
        for (int k = 0; k < 3; k++) xf[k] = ld(f + k * N, plane(zf) + r0);
      }
    }
  };
  auto store_c = [&]() {
#pragma unroll
    for (int c = 0; c < NC; c++) sC[c * HP + p0] = xc0[c];
    if (halo) {
#pragma unroll
      for (int c = 0; c < NC; c++) sC[c * HP + p1] = xc1[c];
    }
  };
  auto store_u = [&](int slot) {
#pragma unroll
    for (int k = 0; k < 3; k++) sU[(slot * 3 + k) * HP + p0] = xu0[k];
    if (halo) {
#pragma unroll
      for (int k = 0; k < 3; k++) sU[(slot * 3 + k) * HP + p1] = xu1[k];
    }
  };
  // -z modulus rows: centre moduli of the previous plane
  R cprev[NC];
  {
    const unsigned o = plane(zs - 1);
#pragma unroll
    for (int c = 0; c < NC; c++) cprev[c] = ld(C + c * SC, o + r0);
  }
  int sm = 0, s0 = 1, sp1 = 2;   // LDS slots of the displacement planes z-1, z, z+1
  issue(zs, zs - 1, zs, 3);
  store_u(sm);
  issue(zs, zs, zs, 3);
  store_u(s0);
  issue(zs, zs + 1, zs, 3);
  store_u(sp1);
  for (int q = 0; q < 3; q++) issue(zs, zs, zs, q);
  store_c();
  __syncthreads();
  // carried to the next step: rows through the y terms, the -z term, centre
  // displacement, diagonal, strain, right-hand side
  R cA[3], cM[3], cu[3], cd[3], ce[NV], cf[3];
  float cdf[3];   // FP32 diagonal (JZ)
  auto finish = [&](int zp, const R *cz) {   // cz: moduli of plane zp + 1 at the node
    const unsigned o = plane(zp) + r0;
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      const int Iv = vslot<3>(i, 2);
      R sg = R(0);
#pragma unroll
      for (int J = 0; J < NV; J++) sg += cz[utri(NV, Iv, J)] * ce[J];
      R a = cA[i];
      a += sg * i2h[2];
      a += -cM[i] * i2h[2];
      if (inbox) {
        TO *__restrict__ oi = (TO *)((char *)(out + i * N) + o * (unsigned)sizeof(TO));
        if constexpr (MODE == MODE_APPLY) {
          *oi = TO(a);
        } else {
          const R r = cf[i] - a;
          *oi = MODE == MODE_RESID ? TO(r) : TO(cu[i] + omega * r / cd[i]);
          nrm += double(r) * double(r);
          if constexpr (JZ) {
            if (xz) {
              const float r32 = TO(r);
              *(float *)((char *)(xz + i * N) + o * 4u) = omegaf * r32 / cdf[i];
            }
          }
        }
      }
    }
    if (partial)
      block_sum_256(nrm, partial + sp.sblocks + ((long long)(zp - sp.lo[2]) * sp.nty + cy) * sp.ntx + cx);
  };
  // Order of the next plane's load groups (measured): FP64 issues the
  // displacement and right-hand side with the first moduli and the halo
  // moduli last, after the y rows; FP32 issues the halo moduli after the
  // centre rows and the displacement and right-hand side last.
  constexpr bool UF_FIRST = sizeof(R) == 8;
  for (int z = zs; z < ze; z++) {
    const int zc = z + 1, zu = z + 2 <= ze ? z + 2 : ze;
    if constexpr (UF_FIRST) issue(zc, zu, z, 3);
    issue(zc, zu, z, 0);
    __builtin_amdgcn_sched_barrier(0);
    R uc[3], up[3][3], um[3][3], upp[3][3], upm[3][3], ump[3][3], umm[3][3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const R *U0 = sU + (s0 * 3 + k) * HP, *Um = sU + (sm * 3 + k) * HP, *Up = sU + (sp1 * 3 + k) * HP;
      uc[k] = U0[p0];
      up[k][0] = U0[p0 + 1];
      um[k][0] = U0[p0 - 1];
      up[k][1] = U0[p0 + HX];
      um[k][1] = U0[p0 - HX];
      up[k][2] = Up[p0];
      um[k][2] = Um[p0];
      // mixed pairs (0,1) (0,2) (1,2)
      upp[k][0] = U0[p0 + 1 + HX];
      upm[k][0] = U0[p0 + 1 - HX];
      ump[k][0] = U0[p0 - 1 + HX];
      umm[k][0] = U0[p0 - 1 - HX];
      upp[k][1] = Up[p0 + 1];
      upm[k][1] = Um[p0 + 1];
      ump[k][1] = Up[p0 - 1];
      umm[k][1] = Um[p0 - 1];
      upp[k][2] = Up[p0 + HX];
      upm[k][2] = Um[p0 + HX];
      ump[k][2] = Up[p0 - HX];
      umm[k][2] = Um[p0 - HX];
    }
    R G[3][3], H[3][3][3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
#pragma unroll
      for (int j = 0; j < 3; j++) {
        G[k][j] = (up[k][j] - um[k][j]) * i2h[j];
        H[k][j][j] = (up[k][j] - R(2) * uc[k] + um[k][j]) * ih2[j];
      }
      constexpr int PJ[3] = {0, 0, 1}, PL[3] = {1, 2, 2};
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const int j = PJ[q], l = PL[q];
        R v = ((upp[k][q] - upm[k][q]) - (ump[k][q] - umm[k][q])) * (i2h[j] * i2h[l]);
        H[k][j][l] = v;
        H[k][l][j] = v;
      }
    }
    R e[NV];
#pragma unroll
    for (int a = 0; a < 3; a++) e[a] = G[a][a];
    e[3] = G[1][2] + G[2][1];
    e[4] = G[0][2] + G[2][0];
    e[5] = G[0][1] + G[1][0];
    __builtin_amdgcn_sched_barrier(0);
    issue(zc, zu, z, 1);
    __builtin_amdgcn_sched_barrier(0);
    R cc[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) cc[c] = sC[c * HP + p0];
    if (z > zs) finish(z - 1, cc);
    R acc[3], dg[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      R a2 = R(0), d2 = R(0);
#pragma unroll
      for (int j = 0; j < 3; j++) {
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
          for (int l = 0; l < 3; l++) a2 += cc[utri(NV, vslot<3>(i, j), vslot<3>(k, l))] * H[k][j][l];
        d2 += cc[utri(NV, vslot<3>(i, j), vslot<3>(i, j))] * ih2[j];
      }
      acc[i] = a2;
      dg[i] = R(-2) * d2;
    }
    if constexpr (!UF_FIRST) {
      __builtin_amdgcn_sched_barrier(0);
      issue(zc, zu, z, 2);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < 2; j++) {   // x and y modulus rows of the LDS neighbours
      if (j == 1 && !UF_FIRST) {
        __builtin_amdgcn_sched_barrier(0);
        issue(zc, zu, z, 3);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int s = 0; s < 2; s++) {
        const int dp = j == 0 ? (s == 0 ? 1 : -1) : (s == 0 ? HX : -HX);
#pragma unroll
        for (int i = 0; i < 3; i++) {
          const int Iv = vslot<3>(i, j);
          R sg = R(0);
#pragma unroll
          for (int J = 0; J < NV; J++) sg += sC[utri(NV, Iv, J) * HP + p0 + dp] * e[J];
          acc[i] += (s == 0 ? sg : -sg) * i2h[j];
        }
      }
    }
    if constexpr (UF_FIRST) {
      __builtin_amdgcn_sched_barrier(0);
      issue(zc, zu, z, 2);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
      const int Iv = vslot<3>(i, 2);
      R sg = R(0);
#pragma unroll
      for (int J = 0; J < NV; J++) sg += cprev[utri(NV, Iv, J)] * e[J];
      cM[i] = sg;
      cA[i] = acc[i];
      cu[i] = uc[i];
      cd[i] = dg[i];
      if constexpr (JZ) {   // interior-row diagonal of diag_at in FP32 from the rounded moduli
        float s2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 3; j++)
          s2 += float(cc[utri(NV, vslot<3>(i, j), vslot<3>(i, j))]) * float(1.0 / (g.h[j] * g.h[j]));
        cdf[i] = -2.0f * s2;
      }
    }
#pragma unroll
    for (int a = 0; a < NV; a++) ce[a] = e[a];
#pragma unroll
    for (int c = 0; c < NC; c++) cprev[c] = cc[c];
    __syncthreads();
    if constexpr (MODE != MODE_APPLY) {
#pragma unroll
      for (int k = 0; k < 3; k++) cf[k] = xf[k];
    }
    if (z + 1 < ze) {
      store_c();
      store_u(sm);
      const int t0 = sm;
      sm = s0;
      s0 = sp1;
      sp1 = t0;
    }
    __syncthreads();
  }
  R cz[NC];
  const unsigned o = plane(ze);
#pragma unroll
  for (int c = 0; c < NC; c++) cz[c] = ld(C + c * SC, o + r0);
  finish(ze - 1, cz);
}

// z-marching pass over an isotropic 3D level.  The workgroup keeps a ring
// of three planes (z-1, z, z+1) of lambda, mu and the displacement in LDS,
// each with the one-node x/y halo, and computes plane z with interior_rows
// itself, addressing the ring by node index plus per-axis offsets (x: 1, y:
// a row, z: the distance between ring slots), so every row is the tile
// kernel's arithmetic on the same values, bit for bit.  Per node and plane
// about 13 global loads (lambda, mu, displacement of the next plane with its
// halo, right-hand side) instead of about 74.  Norm partials go to the tile
// kernel's 64 x 4 slots.  LDS slot layout: ((slot * 3 + component) * HP +
// position), lambda and mu in components 0 and 1 of the moduli ring.  xz
// (FP64 residual to FP32 only): also the FP32 cycle's first sweep from zero,
// as in zm_column.
template <typename R, int MODE, typename TO>
__device__ __forceinline__ void zm_column_iso(const Geom &g, const Split &sp, const R *__restrict__ C,
                                              const R *__restrict__ u, const R *__restrict__ f, TO *__restrict__ out,
                                              R omega, double *__restrict__ partial, int nzc, unsigned w,
                                              R *__restrict__ sC, R *__restrict__ sU, float *__restrict__ xz = nullptr,
                                              float omegaf = 0.0f) {
  constexpr bool JZ = MODE == MODE_RESID && std::is_same<R, double>::value && std::is_same<TO, float>::value;
  constexpr int TX = BX, TY = BY, HX = ZM_HX, HY = ZM_HY, HP = ZM_HP, NH = ZM_NH, PL = 3 * HP;
  constexpr int HW = (NH + 63) / 64;
  const int tx = threadIdx.x, ty = threadIdx.y, t = ty * TX + tx;
  const int wave = __builtin_amdgcn_readfirstlane(ty);
  const unsigned nwg = (unsigned)sp.ntx * sp.nty * nzc;
  const unsigned L = nwg % kXCD == 0 ? (w % kXCD) * (nwg / kXCD) + w / kXCD : w;
  const int chunk = L % nzc, col = L / nzc;
  const int cx = col % sp.ntx, cy = col / sp.ntx;
  const int x0 = sp.lo[0] + cx * TX, y0 = sp.lo[1] + cy * TY;
  const int nz = sp.hi[2] - sp.lo[2] + 1;
  const int zs = sp.lo[2] + (int)((long long)nz * chunk / nzc);
  const int ze = sp.lo[2] + (int)((long long)nz * (chunk + 1) / nzc);
  const int m0 = g.m[0], m1 = g.m[1], m2 = g.m[2];
  auto fix = [](int c, int m, int per) {
    if (per) {
      c %= m;
      return c < 0 ? c + m : c;
    }
    return c < 0 ? 0 : (c > m - 1 ? m - 1 : c);
  };
  const bool inbox = x0 + tx <= sp.hi[0] && y0 + ty <= sp.hi[1];
  const int p0 = (ty + 1) * HX + tx + 1;
  const unsigned r0 = (unsigned)fix(y0 + ty, m1, g.per[1]) * m0 + fix(x0 + tx, m0, g.per[0]);
  int p1 = p0;
  unsigned r1 = r0;
  if (t < NH) {
    int hx, hy;
    if (t < HX) {
      hy = 0;
      hx = t;
    } else if (t < 2 * HX) {
      hy = HY - 1;
      hx = t - HX;
    } else {
      const int q = t - 2 * HX;
      hy = 1 + q / 2;
      hx = (q & 1) ? HX - 1 : 0;
    }
    p1 = hy * HX + hx;
    r1 = (unsigned)fix(y0 + hy - 1, m1, g.per[1]) * m0 + fix(x0 + hx - 1, m0, g.per[0]);
  }
  const bool halo = wave < HW;
  const unsigned P = (unsigned)m0 * m1;
  const long long N = g.N, SC = g.SC;
  auto plane = [&](int z) {
    if (g.per[2]) z = z < 0 ? z + m2 : (z >= m2 ? z - m2 : z);
    return (unsigned)z * P;
  };
  R i2h[3], ih2[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    i2h[a] = R(0.5 / g.h[a]);
    ih2[a] = R(1.0 / (g.h[a] * g.h[a]));
  }
  // a plane in flight: lambda, mu, displacement at the node and the halo position
  R xc0[2], xc1[2], xu0[3], xu1[3], xf[3];
  auto issue = [&](int zn) {
    const unsigned o = plane(zn);
#pragma unroll
    for (int c = 0; c < 2; c++) xc0[c] = ld(C + c * SC, o + r0);
#pragma unroll
    for (int k = 0; k < 3; k++) xu0[k] = ld(u + k * N, o + r0);
    if (halo) {
#pragma unroll
      for (int c = 0; c < 2; c++) xc1[c] = ld(C + c * SC, o + r1);
#pragma unroll
      for (int k = 0; k < 3; k++) xu1[k] = ld(u + k * N, o + r1);
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int c = 0; c < 2; c++) sC[slot * PL + c * HP + p0] = xc0[c];
#pragma unroll
    for (int k = 0; k < 3; k++) sU[slot * PL + k * HP + p0] = xu0[k];
    if (halo) {
#pragma unroll
      for (int c = 0; c < 2; c++) sC[slot * PL + c * HP + p1] = xc1[c];
#pragma unroll
      for (int k = 0; k < 3; k++) sU[slot * PL + k * HP + p1] = xu1[k];
    }
  };
  struct RingU {   // displacement accessor on the LDS ring: component k at index i
    const R *s;
    __device__ __forceinline__ R operator()(int k, int i) const { return s[k * HP + i]; }
  };
  int sm = 0, s0 = 1, sp1 = 2;   // ring slots of planes z-1, z, z+1
  issue(zs - 1);
  store(sm);
  issue(zs);
  store(s0);
  issue(zs + 1);
  store(sp1);
  __syncthreads();
  for (int z = zs; z < ze; z++) {
    if (z + 1 < ze) issue(z + 2);
    if constexpr (MODE != MODE_APPLY) {
#pragma unroll
      for (int k = 0; k < 3; k++) xf[k] = ld(f + k * N, plane(z) + r0);
    }
    const int n = s0 * PL + p0;
    const int om[3] = {-1, -HX, (sm - s0) * PL}, op[3] = {1, HX, (sp1 - s0) * PL};
    R acc[3], dg[3], uc[3];
    interior_rows<3, MOD_ISO, R, RingU, int>(sC, HP, RingU{sU}, n, om, op, i2h, ih2, acc, dg, nullptr, 0, nullptr, uc);
    double nrm = 0.0;
    const unsigned o = plane(z) + r0;
    float cdf[3];   // JZ: the interior-row diagonal of k_jacobi_zero<float> (diag_at on the rounded moduli)
    if constexpr (JZ) {
      if (xz && inbox) {   // the same diag_at, reading lambda and mu from the ring (component stride HP)
        Geom gr = g;
        gr.SC = HP;
        const int pn[3] = {x0 + tx, y0 + ty, z};
        diag_at<3, MOD_ISO, float, double>(gr, sC, (long long)n, pn, ROW_INT, cdf);
      }
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
      if (inbox) {
        TO *__restrict__ oi = (TO *)((char *)(out + i * N) + o * (unsigned)sizeof(TO));
        if constexpr (MODE == MODE_APPLY) {
          *oi = TO(acc[i]);
        } else {
          const R r = xf[i] - acc[i];
          *oi = MODE == MODE_RESID ? TO(r) : TO(uc[i] + omega * r / dg[i]);
          nrm += double(r) * double(r);
          if constexpr (JZ) {
            if (xz) {
              const float r32 = TO(r);
              *(float *)((char *)(xz + i * N) + o * 4u) = omegaf * r32 / cdf[i];
            }
          }
        }
      }
    }
    if (partial)
      block_sum_256(nrm, partial + sp.sblocks + ((long long)(z - sp.lo[2]) * sp.nty + cy) * sp.ntx + cx);
    __syncthreads();
    if (z + 1 < ze) {
      store(sm);
      const int t0 = sm;
      sm = s0;
      s0 = sp1;
      sp1 = t0;
    }
    __syncthreads();
  }
}

// z-marching interior workgroups first (nwg of them), then the shell blocks
// of body_stencil; one launch covers the level.  Anisotropic FP64 needs more
// than 256 registers (one workgroup per CU, which its 95 KB of LDS implies
// anyway); FP32 fits two workgroups per CU.  The isotropic pass (57 KB of
// LDS in FP64, about 210 registers) fits two per CU, four in FP32.
template <typename R, int MODE, typename TO, int K = MOD_ANISO>
__global__ __launch_bounds__(256, sizeof(R) == 8 ? 1 : 2) void k_stencil_zm(Geom g, const R *__restrict__ C,
                                                                           const R *__restrict__ u,
                                                                           const R *__restrict__ f,
                                                                           TO *__restrict__ out, R omega,
                                                                           double *__restrict__ partial,
                                                                           const Ctl *__restrict__ ctl, int nzc,
                                                                           float *__restrict__ xz = nullptr,
                                                                           float omegaf = 0.0f) {
  if (skip(ctl)) return;
  __shared__ R sC[(K == MOD_ISO ? 9 : 21) * ZM_HP];
  __shared__ R sU[9 * ZM_HP];
  const Split sp = split_of(g);
  const unsigned nwg = (unsigned)sp.ntx * sp.nty * nzc;
  if (blockIdx.x < nwg) {
    if constexpr (K == MOD_ISO)
      zm_column_iso<R, MODE, TO>(g, sp, C, u, f, out, omega, partial, nzc, blockIdx.x, sC, sU, xz, omegaf);
    else
      zm_column<R, MODE, TO>(g, sp, C, u, f, out, omega, partial, nzc, blockIdx.x, sC, sU, xz, omegaf);
  } else {
    const long long t = blockIdx.x - nwg;
    body_stencil<3, K, R, MODE, TO>(g, C, u, f, out, omega, partial ? partial + t : nullptr, t);
    if constexpr (MODE == MODE_RESID && std::is_same<R, double>::value && std::is_same<TO, float>::value) {
      if (xz) {   // first FP32 sweep from zero on the shell nodes of this block (as k_jacobi_zero<float>)
        const long long s = t * 256 + threadIdx.x + BX * threadIdx.y;
        if (s < sp.shell) {
          int p[3];
          shell_node(g, sp, s, p);
          const long long n = ((long long)p[2] * g.m[1] + p[1]) * g.m[0] + p[0];
          const int cls = row_class(g, p);
          float dg[3];
          diag_at<3, K, float, double>(g, C, n, p, cls, dg);
#pragma unroll
          for (int i = 0; i < 3; i++) {
            const long long q = i * g.N + n;
            const float f32 = out[q];   // this thread's own store
            xz[q] = (cls == ROW_DIR) ? f32 : omegaf * f32 / dg[i];
          }
        }
      }
    }
  }
}

// u += e (FP32 correction into the FP64 iterate), pointwise.
__global__ __launch_bounds__(256) void k_add_correction(long long n, double *__restrict__ u, const float *__restrict__ e,
                                                       const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    u[i] += double(e[i]);
}

// First sweep from a zero initial guess: out = omega f / diag (Dirichlet: f).
template <int D, int K, typename R, int TX = BX, int TY = BY>
__device__ __forceinline__ void body_jacobi_zero(const Geom &g, const R *__restrict__ C, const R *__restrict__ f,
                                                 R *__restrict__ out, R omega, int tx, int ty, int tz,
                                                 const unsigned char *__restrict__ vm = nullptr,
                                                 const int lx = threadIdx.x, const int ly = threadIdx.y) {
  const int x = tx * TX + lx, y = ty * TY + ly, z = tz;
  if (x >= g.m[0] || y >= g.m[1]) return;
  const long long n = ((long long)z * g.m[1] + y) * g.m[0] + x;
  const int p[3] = {x, y, z};
  const int cls = (vm && !vm[n]) ? ROW_DIR : row_class(g, p);
  R dg[D];
  diag_at<D, K, R>(g, C, n, p, cls, dg);
#pragma unroll
  for (int i = 0; i < D; i++) {
    const long long q = i * g.N + n;
    out[q] = (cls == ROW_DIR) ? f[q] : omega * f[q] / dg[i];
  }
}

template <int D, int K, typename R>
__global__ __launch_bounds__(256) void k_jacobi_zero(Geom g, const R *__restrict__ C, const R *__restrict__ f,
                                                     R *__restrict__ out, R omega, const Ctl *__restrict__ ctl,
                                                     const unsigned char *__restrict__ vm,
                                                     const int *__restrict__ act) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_in(act, g.m[0], g.m[1], tx_, ty_, tz_);
  body_jacobi_zero<D, K, R>(g, C, f, out, omega, tx_, ty_, tz_, vm);
}

// Per-axis full-weighting weights and fine offsets of coarse node P (fine
// node pf = 2P): [1/4, 1/2, 1/4] on an axis along which P is not on an end,
// else (0, 1, 0) (only the coincident fine node).  Every 3^D stencil point is
// then summed, the excluded ones with weight 0 and offset 0, so all loads
// issue at once; the sum over the included points is unchanged (exact zeros).
template <typename R>
__device__ __forceinline__ void fw_weights(const Geom &gc, const Geom &gf, const int P[3], const int pf[3], int dim,
                                           R wt[3][3], long long off[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    off[a][0] = off[a][1] = off[a][2] = 0;
    wt[a][0] = wt[a][2] = R(0);
    wt[a][1] = R(1);
    if (a < dim && end_of(gc, a, P[a]) == 0) {
      wt[a][0] = wt[a][2] = R(0.25);
      wt[a][1] = R(0.5);
      off[a][0] = shift(gf, a, pf[a], -1);
      off[a][2] = shift(gf, a, pf[a], 1);
    }
  }
}

// Full-weighting restriction (tensor product of [1/4, 1/2, 1/4]); along an
// axis on whose end the coarse node sits only the coincident fine node
// enters; Dirichlet coarse rows get 0.
template <int D, typename RI, typename RO, int TX = BX, int TY = BY>
__device__ __forceinline__ void body_restrict(const Geom &gf, const Geom &gc, const RI *__restrict__ rf,
                                              RO *__restrict__ fc, int tx, int ty, int tz,
                                              const int lx = threadIdx.x, const int ly = threadIdx.y) {
  const int x = tx * TX + lx, y = ty * TY + ly, z = tz;
  if (x >= gc.m[0] || y >= gc.m[1]) return;
  const long long nc = ((long long)z * gc.m[1] + y) * gc.m[0] + x;
  const int P[3] = {x, y, z};
  const int cls = row_class(gc, P);
  if (cls == ROW_DIR) {
    for (int i = 0; i < D; i++) fc[i * gc.N + nc] = RO(0);
    return;
  }
  const int pf[3] = {2 * x, 2 * y, 2 * z};
  const long long nf = ((long long)pf[2] * gf.m[1] + pf[1]) * gf.m[0] + pf[0];
  RI wt[3][3];
  long long off[3][3];
  fw_weights<RI>(gc, gf, P, pf, D, wt, off);
  RI acc[D];
#pragma unroll
  for (int i = 0; i < D; i++) acc[i] = RI(0);
  constexpr int ZR = D == 3 ? 1 : 0;
#pragma unroll
  for (int oz = -ZR; oz <= ZR; oz++)
#pragma unroll
    for (int oy = -1; oy <= 1; oy++)
#pragma unroll
      for (int ox = -1; ox <= 1; ox++) {
        const RI w = wt[0][ox + 1] * wt[1][oy + 1] * wt[2][oz + 1];
        const long long q = nf + off[0][ox + 1] + off[1][oy + 1] + off[2][oz + 1];
#pragma unroll
        for (int i = 0; i < D; i++) acc[i] += w * rf[i * gf.N + q];
      }
#pragma unroll
  for (int i = 0; i < D; i++) fc[i * gc.N + nc] = RO(acc[i]);
}

template <int D, typename RI, typename RO, int TX = BX, int TY = BY>
__global__ __launch_bounds__(TX * TY) void k_restrict(Geom gf, Geom gc, const RI *__restrict__ rf,
                                                      RO *__restrict__ fc, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  body_restrict<D, RI, RO, TX, TY>(gf, gc, rf, fc, tx_, ty_, tz_);
}

// Restriction fused with the coarse level's first Jacobi sweep from zero
// (x = omega f / diag, Dirichlet rows x = f = 0): the same values as
// k_restrict followed by k_jacobi_zero, one launch instead of two.  The
// diagonal's moduli loads are issued with the fine residual's, so the two
// latencies overlap.
template <int D, int K, typename R, int TX = BX, int TY = BY>
__global__ __launch_bounds__(TX * TY) void k_restrict_jz(Geom gf, Geom gc, const R *__restrict__ rf, R *__restrict__ fc,
                                                     const R *__restrict__ Cc, R *__restrict__ xc, R omega,
                                                     const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  const int x = tx_ * TX + threadIdx.x, y = ty_ * TY + threadIdx.y, z = tz_;
  if (x >= gc.m[0] || y >= gc.m[1]) return;
  const long long nc = ((long long)z * gc.m[1] + y) * gc.m[0] + x;
  const int P[3] = {x, y, z};
  const int cls = row_class(gc, P);
  if (cls == ROW_DIR) {
#pragma unroll
    for (int i = 0; i < D; i++) {
      fc[i * gc.N + nc] = R(0);
      xc[i * gc.N + nc] = R(0);
    }
    return;
  }
  R dg[D];
  diag_at<D, K, R>(gc, Cc, nc, P, cls, dg);
  const int pf[3] = {2 * x, 2 * y, 2 * z};
  const long long nf = ((long long)pf[2] * gf.m[1] + pf[1]) * gf.m[0] + pf[0];
  R wt[3][3];
  long long off[3][3];
  fw_weights<R>(gc, gf, P, pf, D, wt, off);
  R acc[D];
#pragma unroll
  for (int i = 0; i < D; i++) acc[i] = R(0);
  constexpr int ZR = D == 3 ? 1 : 0;
#pragma unroll
  for (int oz = -ZR; oz <= ZR; oz++)
#pragma unroll
    for (int oy = -1; oy <= 1; oy++)
#pragma unroll
      for (int ox = -1; ox <= 1; ox++) {
        const R w = wt[0][ox + 1] * wt[1][oy + 1] * wt[2][oz + 1];
        const long long q = nf + off[0][ox + 1] + off[1][oy + 1] + off[2][oz + 1];
#pragma unroll
        for (int i = 0; i < D; i++) acc[i] += w * rf[i * gf.N + q];
      }
#pragma unroll
  for (int i = 0; i < D; i++) {
    fc[i * gc.N + nc] = acc[i];
    xc[i * gc.N + nc] = omega * acc[i] / dg[i];
  }
}

// u_fine += bilinear/trilinear interpolation of the coarse correction;
// Dirichlet fine rows untouched.
template <int D, typename RC, typename RF, int TX = BX, int TY = BY>
__device__ __forceinline__ void body_prolong(const Geom &gc, const Geom &gf, const RC *__restrict__ ec,
                                             RF *__restrict__ uf, int tx, int ty, int tz,
                                             const int lx = threadIdx.x, const int ly = threadIdx.y) {
  const int x = tx * TX + lx, y = ty * TY + ly, z = tz;
  if (x >= gf.m[0] || y >= gf.m[1]) return;
  const long long n = ((long long)z * gf.m[1] + y) * gf.m[0] + x;
  const int p[3] = {x, y, z};
  if (row_class(gf, p) == ROW_DIR) return;
  const int b[3] = {x >> 1, y >> 1, z >> 1};
  const long long nb = ((long long)b[2] * gc.m[1] + b[1]) * gc.m[0] + b[0];
  // per axis: (1/2, 1/2) at b, b+1 for an odd fine coordinate, else (1, 0);
  // all 2^D corners are summed (weight 0 and offset 0 for the unused ones)
  RC wt[3][2];
  long long o1[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const bool odd = a < D && (p[a] & 1);
    wt[a][0] = odd ? RC(0.5) : RC(1);
    wt[a][1] = odd ? RC(0.5) : RC(0);
    o1[a] = odd ? shift(gc, a, b[a], 1) : 0;
  }
  RC acc[D];
#pragma unroll
  for (int i = 0; i < D; i++) acc[i] = RC(0);
  constexpr int ZC = D == 3 ? 2 : 1;
#pragma unroll
  for (int cz = 0; cz < ZC; cz++)
#pragma unroll
    for (int cy = 0; cy < 2; cy++)
#pragma unroll
      for (int cx = 0; cx < 2; cx++) {
        const RC w = wt[0][cx] * wt[1][cy] * wt[2][cz];
        const long long q = nb + (cx ? o1[0] : 0) + (cy ? o1[1] : 0) + (cz ? o1[2] : 0);
#pragma unroll
        for (int i = 0; i < D; i++) acc[i] += w * ec[i * gc.N + q];
      }
#pragma unroll
  for (int i = 0; i < D; i++) uf[i * gf.N + n] += RF(acc[i]);
}

template <int D, typename RC, typename RF, int TX = BX, int TY = BY>
__global__ __launch_bounds__(TX * TY) void k_prolong_add(Geom gc, Geom gf, const RC *__restrict__ ec,
                                                         RF *__restrict__ uf, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  body_prolong<D, RC, RF, TX, TY>(gc, gf, ec, uf, tx_, ty_, tz_);
}

// 3D interpolation with the coarse values of a fine TX x TY tile staged in
// LDS: the tile needs coarse x in [x0/2, x0/2 + TX/2], y in [y0/2, y0/2 +
// TY/2] and planes z/2, z/2 + 1 (198 nodes for 64 x 4), loaded once by the
// threads of the tile instead of 8 loads per component by every fine node.  Coarse coordinates
// wrap on periodic axes and clamp otherwise (clamped values only enter with
// weight 0 or for fine nodes outside the grid).  The sum per fine node is
// that of body_prolong, term by term.
template <typename RC, typename RF, int TX = BX, int TY = BY>
__global__ __launch_bounds__(TX * TY) void k_prolong3_lds(Geom gc, Geom gf, const RC *__restrict__ ec,
                                                          RF *__restrict__ uf, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  constexpr int CX = TX / 2 + 1, CY = TY / 2 + 1, CP = CX * CY * 2;
  __shared__ RC sE[3][CP];
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  const int x0 = tx_ * TX, y0 = ty_ * TY, z = tz_;
  for (int t = threadIdx.x + TX * threadIdx.y; t < CP; t += TX * TY) {
    const int cx = t % CX, cy = (t / CX) % CY, cz = t / (CX * CY);
    int c[3] = {x0 / 2 + cx, y0 / 2 + cy, z / 2 + cz};
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (gc.per[a]) c[a] %= gc.m[a];
      else c[a] = c[a] > gc.m[a] - 1 ? gc.m[a] - 1 : c[a];
    }
    const long long q = ((long long)c[2] * gc.m[1] + c[1]) * gc.m[0] + c[0];
#pragma unroll
    for (int i = 0; i < 3; i++) sE[i][t] = ec[i * gc.N + q];
  }
  __syncthreads();
  const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
  if (x >= gf.m[0] || y >= gf.m[1]) return;
  const int p[3] = {x, y, z};
  if (row_class(gf, p) == ROW_DIR) return;
  const long long n = ((long long)z * gf.m[1] + y) * gf.m[0] + x;
  // local coarse base (threadIdx.x >> 1, threadIdx.y >> 1, 0); per axis the
  // weights (1/2, 1/2) for an odd fine coordinate, else (1, 0)
  RC wt[3][2];
  int o1[3];
  const int st[3] = {1, CX, CX * CY};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const bool odd = p[a] & 1;
    wt[a][0] = odd ? RC(0.5) : RC(1);
    wt[a][1] = odd ? RC(0.5) : RC(0);
    o1[a] = odd ? st[a] : 0;
  }
  const int lb = (threadIdx.x >> 1) + CX * (threadIdx.y >> 1);
  RC acc[3] = {RC(0), RC(0), RC(0)};
#pragma unroll
  for (int cz = 0; cz < 2; cz++)
#pragma unroll
    for (int cy = 0; cy < 2; cy++)
#pragma unroll
      for (int cx = 0; cx < 2; cx++) {
        const RC w = wt[0][cx] * wt[1][cy] * wt[2][cz];
        const int q = lb + (cx ? o1[0] : 0) + (cy ? o1[1] : 0) + (cz ? o1[2] : 0);
#pragma unroll
        for (int i = 0; i < 3; i++) acc[i] += w * sE[i][q];
      }
#pragma unroll
  for (int i = 0; i < 3; i++) uf[i * gf.N + n] += RF(acc[i]);
}

// Coarse-level moduli: full weighting of each stored component, injection
// along an axis on whose end the coarse node sits.
// Grid: x and y tiles of the coarse level, blockIdx.z = plane + m2 * component.
template <typename R>
__global__ __launch_bounds__(256) void k_coarsen(Geom gf, Geom gc, int nc, const R *__restrict__ Cf, R *__restrict__ Cc) {
  const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
  const int z = blockIdx.z % gc.m[2], c = blockIdx.z / gc.m[2];
  if (x >= gc.m[0] || y >= gc.m[1] || c >= nc) return;
  const long long n = ((long long)z * gc.m[1] + y) * gc.m[0] + x;
  const int P[3] = {x, y, z};
  const int pf[3] = {2 * x, 2 * y, 2 * z};
  const long long nf = ((long long)pf[2] * gf.m[1] + pf[1]) * gf.m[0] + pf[0];
  R wt[3][3];
  long long off[3][3];
  fw_weights<R>(gc, gf, P, pf, gc.dim, wt, off);
  const R *__restrict__ F = Cf + c * gf.SC + nf;
  R acc = R(0);
#pragma unroll
  for (int oz = -1; oz <= 1; oz++)
#pragma unroll
    for (int oy = -1; oy <= 1; oy++)
#pragma unroll
      for (int ox = -1; ox <= 1; ox++) {
        const R w = wt[0][ox + 1] * wt[1][oy + 1] * wt[2][oz + 1];
        acc += w * F[off[0][ox + 1] + off[1][oy + 1] + off[2][oz + 1]];
      }
  Cc[c * gc.SC + n] = acc;
}

// Face data of all faces (d components per face node, normal axis extent 1).
struct Faces {
  const double *p[6];
};

__device__ __forceinline__ double face_val(const Geom &g, const Faces &F, int f, const int p[3], int i) {
  const double *a = F.p[f];
  if (!a) return 0.0;
  const int ax = f / 2;
  int q[3] = {p[0], p[1], p[2]}, fm[3] = {g.m[0], g.m[1], g.m[2]};
  q[ax] = 0;
  fm[ax] = 1;
  const long long fn = (long long)fm[0] * fm[1] * fm[2];
  return a[i * fn + ((long long)q[2] * fm[1] + q[1]) * fm[0] + q[0]];
}

// C:E contracted on the last pair: sum_kl C_ijkl E_kl for node moduli c[]
// and symmetric tensor E given by its Voigt-ordered tensor components.
template <int D, int K>
__device__ __forceinline__ double c_dot_e(const double *c, const double *E, int i, int j) {
  double s = 0.0;
  for (int k = 0; k < D; k++)
    for (int l = 0; l < D; l++) s += cfull<D, K, double>(c, i, j, k, l) * E[vslot<D>(k, l)];
  return s;
}

// Right-hand side: interior -b + d_j(C_ijkl eps0_kl) by the product rule
// (= -(D(0) + b), Sec. 2.1.1); traction rows sum_f t0_f + C eps0 n_f;
// Neumann rows the sum of the prescribed normal derivatives of the node's
// Neumann faces; Dirichlet rows u0 of the lowest-numbered Dirichlet face.
template <int D, int K>
__global__ __launch_bounds__(256) void k_rhs(Geom g, const double *__restrict__ C, const double *__restrict__ eps,
                                             const double *__restrict__ b, Faces F, double *__restrict__ f) {
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  const int x = tx_ * BX + threadIdx.x, y = ty_ * BY + threadIdx.y, z = tz_;
  if (x >= g.m[0] || y >= g.m[1]) return;
  constexpr int NC = nmod<D, K>(), NE = nvoigt<D>();
  const long long n = ((long long)z * g.m[1] + y) * g.m[0] + x;
  const int p[3] = {x, y, z};
  const int cls = row_class(g, p);
  double cc[NC], ec[NE];
  for (int c = 0; c < NC; c++) cc[c] = C[c * g.SC + n];
  for (int c = 0; c < NE; c++) ec[c] = eps ? eps[c * g.N + n] : 0.0;
  if (cls == ROW_INT) {   // neighbour moduli and eigenstrain loaded once per axis for all rows
    double acc[D];
#pragma unroll
    for (int i = 0; i < D; i++) acc[i] = b ? 0.0 - b[i * g.N + n] : 0.0;
    if (eps) {
#pragma unroll
      for (int j = 0; j < D; j++) {
        const long long sp = shift(g, j, p[j], 1), sm = shift(g, j, p[j], -1);
        double cp[NC], cm[NC], ep[NE], em[NE];
#pragma unroll
        for (int c = 0; c < NC; c++) {
          cp[c] = C[c * g.SC + n + sp];
          cm[c] = C[c * g.SC + n + sm];
        }
#pragma unroll
        for (int c = 0; c < NE; c++) {
          ep[c] = eps[c * g.N + n + sp];
          em[c] = eps[c * g.N + n + sm];
        }
        const double inv2h = 0.5 / g.h[j];
#pragma unroll
        for (int i = 0; i < D; i++) {
          acc[i] += (c_dot_e<D, K>(cp, ec, i, j) - c_dot_e<D, K>(cm, ec, i, j)) * inv2h;
          acc[i] += (c_dot_e<D, K>(cc, ep, i, j) - c_dot_e<D, K>(cc, em, i, j)) * inv2h;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < D; i++) f[i * g.N + n] = acc[i];
    return;
  }
  for (int i = 0; i < D; i++) {
    double acc = 0.0;
    if (cls == ROW_DIR) {
      for (int fc = 0; fc < 2 * D; fc++) {
        const int e = end_of(g, fc / 2, p[fc / 2]);
        if (((fc & 1) ? e > 0 : e < 0) && g.bc[fc] == BC_DIR) {
          acc = face_val(g, F, fc, p, i);
          break;
        }
      }
    } else if (cls == ROW_NEU) {
      for (int a = 0; a < D; a++) {
        const int na = neumann_normal(g, a, p);
        if (na) acc += face_val(g, F, 2 * a + (na > 0), p, i);
      }
    } else {
      for (int fc = 0; fc < 2 * D; fc++) {
        const int a = fc / 2;
        const int e = end_of(g, a, p[a]);
        if (!((fc & 1) ? e > 0 : e < 0)) continue;
        acc += face_val(g, F, fc, p, i);
        if (eps) acc += double(e) * c_dot_e<D, K>(cc, ec, i, a);
      }
    }
    f[i * g.N + n] = acc;
  }
}

// Von Mises stress sqrt(3/2 S:S) of a 3D Voigt stress [11,22,33,23,31,12]
// (Sec. 4.3), S the deviator: the off-diagonal entries appear twice in S:S.
__global__ __launch_bounds__(256) void k_von_mises(long long n, const double *__restrict__ sig,
                                                   double *__restrict__ svm) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double s11 = sig[i], s22 = sig[n + i], s33 = sig[2 * n + i];
  const double s23 = sig[3 * n + i], s31 = sig[4 * n + i], s12 = sig[5 * n + i];
  const double p = (s11 + s22 + s33) / 3.0;
  const double d1 = s11 - p, d2 = s22 - p, d3 = s33 - p;
  const double ss = d1 * d1 + d2 * d2 + d3 * d3 + 2.0 * (s23 * s23 + s31 * s31 + s12 * s12);
  svm[i] = sqrt(1.5 * ss);
}

// Stress sigma_ij = C_ijkl (du_k/dx_l - eps0_kl): central differences, 3-point
// one-sided on non-periodic ends; Voigt output.
template <int D, int K>
__global__ __launch_bounds__(256) void k_stress(Geom g, const double *__restrict__ C, const double *__restrict__ eps,
                                                const double *__restrict__ u, double *__restrict__ sig) {
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  const int x = tx_ * BX + threadIdx.x, y = ty_ * BY + threadIdx.y, z = tz_;
  if (x >= g.m[0] || y >= g.m[1]) return;
  constexpr int NC = nmod<D, K>(), NE = nvoigt<D>();
  const long long n = ((long long)z * g.m[1] + y) * g.m[0] + x;
  const int p[3] = {x, y, z};
  double cc[NC];
  for (int c = 0; c < NC; c++) cc[c] = C[c * g.SC + n];
  double E[NE];   // strain minus eigenstrain, tensor components in Voigt order
  double Gd[D][D];
  for (int l = 0; l < D; l++) {
    const int en = end_of(g, l, p[l]);
    const double h = g.h[l];
    for (int k = 0; k < D; k++) {
      const double *uk = u + k * g.N;
      if (en != 0) {
        const int s = -en;
        const long long s1 = shift(g, l, p[l], s), s2 = shift(g, l, p[l], 2 * s);
        Gd[k][l] = s * (-3.0 * uk[n] + 4.0 * uk[n + s1] - uk[n + s2]) / (2.0 * h);
      } else {
        Gd[k][l] = (uk[n + shift(g, l, p[l], 1)] - uk[n + shift(g, l, p[l], -1)]) / (2.0 * h);
      }
    }
  }
  for (int k = 0; k < D; k++)
    for (int l = k; l < D; l++) {
      const int v = vslot<D>(k, l);
      E[v] = 0.5 * (Gd[k][l] + Gd[l][k]) - (eps ? eps[v * g.N + n] : 0.0);
    }
  for (int i = 0; i < D; i++)
    for (int j = i; j < D; j++) sig[vslot<D>(i, j) * g.N + n] = c_dot_e<D, K>(cc, E, i, j);
}

// Dirichlet lift: u = f on Dirichlet rows, 0 elsewhere.
template <int D>
__global__ __launch_bounds__(256) void k_lift(Geom g, const double *__restrict__ f, double *__restrict__ u) {
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  const int x = tx_ * BX + threadIdx.x, y = ty_ * BY + threadIdx.y, z = tz_;
  if (x >= g.m[0] || y >= g.m[1]) return;
  const long long n = ((long long)z * g.m[1] + y) * g.m[0] + x;
  const int p[3] = {x, y, z};
  const bool dir = row_class(g, p) == ROW_DIR;
  for (int i = 0; i < D; i++) u[i * g.N + n] = dir ? f[i * g.N + n] : 0.0;
}

template <typename A, typename B>
__global__ __launch_bounds__(256) void k_cast(long long n, const A *__restrict__ in, B *__restrict__ out,
                                              const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) out[i] = B(in[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(long long n, T *__restrict__ out, T v) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) out[i] = v;
}

// Sum the norm partials in a fixed order and update the control block.
// `ans` is the buffer index of the iterate whose residual was measured.
__device__ __forceinline__ void body_check(const double *__restrict__ partial, long long nparts, Ctl *ctl, int ans);

__global__ __launch_bounds__(1024) void k_check(const double *__restrict__ partial, long long nparts, Ctl *ctl, int ans) {
  body_check(partial, nparts, ctl, ans);
}

__device__ __forceinline__ void body_check(const double *__restrict__ partial, long long nparts, Ctl *ctl, int ans) {
  if (ctl->done) return;
  double s0 = 0.0, s1 = 0.0;
  long long i = threadIdx.x;
  for (; i + 1024 < nparts; i += 2048) {
    s0 += partial[i];
    s1 += partial[i + 1024];
  }
  if (i < nparts) s0 += partial[i];
  __shared__ double tot;
  block_sum_1024(s0 + s1, &tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = tot;
    ctl->ans = ans;
    if (!(v == v) || v > 1.0e300) {
      ctl->done = 2;
      return;
    }
    if (ctl->r0sq < 0.0) ctl->r0sq = v;
    ctl->rsq = v;
    if (v <= ctl->tol2 * ctl->r0sq) ctl->done = 1;
    else if (ctl->cycles >= ctl->max_cycles) ctl->done = 3;
    else ctl->cycles += 1;
  }
}

// Store the summed partials as the reference norm (warm starts measure
// convergence relative to the Dirichlet lift's residual).
__global__ __launch_bounds__(1024) void k_set_r0(const double *__restrict__ partial, long long nparts, Ctl *ctl) {
  double s = 0.0;
  for (long long i = threadIdx.x; i < nparts; i += 1024) s += partial[i];
  __shared__ double tot;
  block_sum_1024(s, &tot);
  __syncthreads();
  if (threadIdx.x == 0) ctl->r0sq = tot;
}

// ---- coarsest level: dense matrix by unit vectors, Gauss-Jordan inverse ----

// M (n x 2n, row-major) = [A | I] with A the level's D_H.
template <int D, int K>
__global__ __launch_bounds__(256) void k_bottom_assemble(Geom g, const double *__restrict__ C, double *__restrict__ M,
                                                         int nunk) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int q = blockIdx.y;
  if (r >= nunk) return;
  const int i = r / (int)g.N;
  const long long n = r % g.N;
  const int p[3] = {int(n % g.m[0]), int((n / g.m[0]) % g.m[1]), int(n / ((long long)g.m[0] * g.m[1]))};
  const int cls = row_class(g, p);
  double acc[D], dg[D];
  rows_at<D, K, double>(g, C, UnitU<double>{q, g.N}, n, p, cls, acc, dg);
  const long long w = 2LL * nunk;
  M[r * w + q] = acc[i];
  M[r * w + nunk + q] = (r == q) ? 1.0 : 0.0;
}

// Blocked Gauss-Jordan on [A | I] (n x 2n, row stride 2n), panels of b
// columns of the left half.  k_gjb_panel (one workgroup) runs the in-place
// Gauss-Jordan steps with partial pivoting (largest |value| among the rows
// not yet pivoted, lowest index on ties) on the panel's n x b values in LDS.
// Those steps turn the panel into N, the transform they apply to any other
// column x whose rows have been permuted alike: the panel's block rows become
// N_block x_block, every other row i becomes x_i + N_i x_block.  It writes N
// and the row permutation pi (row i of the swapped matrix is row pi[i] of the
// input).  k_gjb_update applies that to every column right of the panel,
// out of place.  Per panel two launches instead of b; the arithmetic is the
// same elimination in another order.  status[0] = 1 on a zero pivot.
constexpr int GJB_LDS = 18432;   // doubles of panel in LDS: n * b <= this

// Panel of b <= B columns in LDS at row stride B; thread t owns column
// t % B of the rows t / B + RS m.
template <int B>
__global__ __launch_bounds__(1024) void k_gjb_panel(const double *__restrict__ W, int n, int k, int b,
                                                    double *__restrict__ Nout, int *__restrict__ pi,
                                                    int *__restrict__ status) {
  constexpr int RS = 1024 / B;   // rows per pass
  __shared__ double Q[GJB_LDS];
  __shared__ double cv[512];   // pivot candidates of threads 0..511
  __shared__ int ci[512];
  __shared__ int sp[1536];   // the permutation (written to pi at the end)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int q = t % B, rg = t / B;
  const bool own = rg < RS && q < b;
  const long long w = 2LL * n;
  constexpr int MR = (1536 + RS - 1) / RS;   // passes of rows (n <= 1536), unrolled so the loads overlap
  if (own) {
#pragma unroll
    for (int m = 0; m < MR; m++) {
      const int i = rg + m * RS;
      if (i < n) Q[i * B + q] = W[(long long)i * w + k + q];
    }
  }
  for (int i = t; i < n; i += 1024) sp[i] = i;
  __syncthreads();
  for (int s = 0; s < b; s++) {
    const int c = k + s;
    // pivot: largest |value| of column s among rows >= c, lowest row on ties;
    // candidates of 512 threads, reduced by one wavefront
    if (t < 512) {
      double best = -1.0;
      int arg = c;
      for (int i = c + t; i < n; i += 512) {
        const double v = fabs(Q[i * B + s]);
        if (v > best) {
          best = v;
          arg = i;
        }
      }
      cv[t] = best;
      ci[t] = arg;
    }
    __syncthreads();
    if (wv == 0) {
      double best = cv[lane];
      int arg = ci[lane];
      for (int h = 1; h < 8; h++) {
        const double v = cv[lane + 64 * h];
        const int i = ci[lane + 64 * h];
        if (v > best || (v == best && i < arg)) {
          best = v;
          arg = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double bv = __shfl_xor(best, o);
        const int bi = __shfl_xor(arg, o);
        if (bv > best || (bv == best && bi < arg)) {
          best = bv;
          arg = bi;
        }
      }
      if (lane == 0) ci[0] = arg;
    }
    __syncthreads();
    const int r = ci[0];
    if (r != c && t < b) {
      const double a = Q[c * B + t];
      Q[c * B + t] = Q[r * B + t];
      Q[r * B + t] = a;
    }
    if (r != c && t == 0) {
      const int a = sp[c];
      sp[c] = sp[r];
      sp[r] = a;
    }
    __syncthreads();
    const double piv = Q[c * B + s];
    if (t == 0 && piv == 0.0) status[0] = 1;
    const double inv = piv != 0.0 ? 1.0 / piv : 0.0;
    // other rows, other columns, with the pivot row scaled by inv
    if (own && q != s) {   // chunks of 8 rows: all reads of a chunk in flight before its writes
      const double rc = Q[c * B + q] * inv;
      constexpr int CH = 8;
#pragma unroll
      for (int m0 = 0; m0 < MR; m0 += CH) {
        double xs[CH], xq[CH];
#pragma unroll
        for (int h = 0; h < CH; h++) {
          const int i = rg + (m0 + h) * RS;
          xs[h] = m0 + h < MR && i < n ? Q[i * B + s] : 0.0;
          xq[h] = m0 + h < MR && i < n ? Q[i * B + q] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < CH; h++) {
          const int i = rg + (m0 + h) * RS;
          if (m0 + h < MR && i < n && i != c) Q[i * B + q] = xq[h] - xs[h] * rc;
        }
      }
    }
    __syncthreads();
    // pivot row scaled, pivot column -value / pivot, 1 / pivot at the pivot
    for (int i = t; i < n; i += 1024)
      if (i != c) Q[i * B + s] = -Q[i * B + s] * inv;
    if (t < b) Q[c * B + t] = t == s ? inv : Q[c * B + t] * inv;
    __syncthreads();
  }
  if (own) {
#pragma unroll
    for (int m = 0; m < MR; m++) {
      const int i = rg + m * RS;
      if (i < n) Nout[(long long)i * b + q] = Q[i * B + q];
    }
  }
  for (int i = t; i < n; i += 1024) pi[i] = sp[i];
}

// Columns j >= k + b of W2 from W: y = the b pivot rows of column j after
// the permutation; block rows N_block y, other rows x_pi[i] + N_i y.  Grid:
// x = 256-column blocks, y = 16-row chunks (loads of a chunk in flight
// together).
constexpr int GJB_ROWS = 16;
__global__ __launch_bounds__(256) void k_gjb_update(const double *__restrict__ W, double *__restrict__ W2, int n,
                                                    int k, int b, const double *__restrict__ N,
                                                    const int *__restrict__ pi) {
  __shared__ double Ns[GJB_ROWS * 16];
  __shared__ int ps[GJB_ROWS];
  const int i0 = blockIdx.y * GJB_ROWS;
  const long long w = 2LL * n;
  for (int e = threadIdx.x; e < GJB_ROWS * b; e += 256) {
    const int i = i0 + e / b;
    Ns[e] = i < n ? N[(long long)i * b + e % b] : 0.0;
  }
  if (threadIdx.x < GJB_ROWS) ps[threadIdx.x] = i0 + (int)threadIdx.x < n ? pi[i0 + threadIdx.x] : 0;
  __syncthreads();
  const long long j = (long long)k + b + (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= w) return;
  double y[16], x[GJB_ROWS];
#pragma unroll
  for (int s = 0; s < 16; s++) y[s] = s < b ? W[(long long)pi[k + s] * w + j] : 0.0;
#pragma unroll
  for (int r = 0; r < GJB_ROWS; r++) {
    const int i = i0 + r;
    x[r] = (i < n && (i < k || i >= k + b)) ? W[(long long)ps[r] * w + j] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < GJB_ROWS; r++) {
    const int i = i0 + r;
    if (i >= n) break;
    double acc = x[r];
#pragma unroll
    for (int s = 0; s < 16; s++)
      if (s < b) acc += Ns[r * b + s] * y[s];
    W2[(long long)i * w + j] = acc;
  }
}

__global__ __launch_bounds__(256) void k_gj_extract(const double *__restrict__ M, int n, double *__restrict__ Ainv) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)n * n) return;
  const long long i = idx / n, j = idx % n;
  Ainv[idx] = M[i * 2LL * n + n + j];
}

// e = A^-1 f in FP64, one wavefront per row.
template <typename RI, typename RO>
__device__ __forceinline__ void body_bottom(const double *__restrict__ Ainv, int n, const RI *__restrict__ f,
                                            RO *__restrict__ e, int tile) {
  const int row = tile * 4 + (int)((threadIdx.x + threadIdx.y * blockDim.x) >> 6);
  const int lane = (threadIdx.x + threadIdx.y * blockDim.x) & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += Ainv[(long long)row * n + j] * double(f[j]);
  s = wave_sum(s);
  if (lane == 0) e[row] = RO(s);
}

template <typename RI, typename RO>
__global__ __launch_bounds__(256) void k_bottom_solve(const double *__restrict__ Ainv, int n, const RI *__restrict__ f,
                                                      RO *__restrict__ e, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  body_bottom<RI, RO>(Ainv, n, f, e, blockIdx.x);
}


}  // namespace emg

// ======================= block-structured AMR coupling =======================
// A refined level is a list of boxes of valid nodes [lo, hi] (even bounds)
// in its own index space; its fields are stored over the bounding box b of
// the boxes grown by one node per side (array extents hi-lo+3), with a byte
// mask vm over that array (1: valid node, the union of the boxes; 0: ghost
// or outside every box).  The array is treated as a level whose faces are
// all Dirichlet and whose masked-out nodes are Dirichlet rows as well, so
// valid nodes (including the coarse/fine boundary layer) are the interior
// rows.  Coarse arrays are addressed with `co`, the global index of their
// array index 0 (0 for the base grid, lo-1 for a refined level).
namespace emg {

struct Box {
  int lo[3], hi[3];   // nodes, fine index space (a level's bounding box)
};

using Mask = const unsigned char *__restrict__;

// coarse node J (global) -> coarse array index, and fine global I -> fine array index
__device__ __forceinline__ long long lin(const Geom &g, int x, int y, int z) {
  return ((long long)z * g.m[1] + y) * g.m[0] + x;
}

// Fine array index of the fine node coincident with coarse node (cx, cy, cz)
// (global indices), for a coarse node under the bounding box b.
template <int D>
__device__ __forceinline__ long long coincident(const Geom &gf, const Box &b, int cx, int cy, int cz) {
  return lin(gf, 2 * cx - b.lo[0] + 1, 2 * cy - b.lo[1] + 1, D == 3 ? 2 * cz - b.lo[2] + 1 : 0);
}

// Covered coarse nodes <- coincident fine values (Sec. 3.2 / App. A:
// phi_c2 = phi_f4).  One thread per coarse node under the bounding box;
// those whose fine node is not valid are not covered.
template <int D, typename R>
__global__ __launch_bounds__(256) void k_inject(Geom gc, int3 co, Geom gf, Box b, Mask vm, const R *__restrict__ uf,
                                                R *__restrict__ uc, int ncomp, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  const int cx = b.lo[0] / 2 + blockIdx.x * BX + threadIdx.x;
  const int cy = b.lo[1] / 2 + blockIdx.y * BY + threadIdx.y;
  const int cz = (D == 3 ? b.lo[2] / 2 : 0) + blockIdx.z;
  if (cx > b.hi[0] / 2 || cy > b.hi[1] / 2 || (D == 3 && cz > b.hi[2] / 2)) return;
  const long long nf = coincident<D>(gf, b, cx, cy, cz);
  if (!vm[nf]) return;
  const long long nc = lin(gc, cx - co.x, cy - co.y, D == 3 ? cz - co.z : 0);
  for (int i = 0; i < ncomp; i++) uc[i * gc.N + nc] = uf[i * gf.N + nf];
}

// Full weighting of a field given on the fine array (moduli, eigenstrain)
// at the covered coarse nodes: coarse levels carry the average of the finer
// level where it exists (Sec. 1).  sf, sc: component strides of af and ac.
template <int D>
__global__ __launch_bounds__(256) void k_average_cf(Geom gc, int3 co, Geom gf, Box b, Mask vm,
                                                    const double *__restrict__ af, double *__restrict__ ac, int ncomp,
                                                    long long sf, long long sc) {
  const int cx = b.lo[0] / 2 + blockIdx.x * BX + threadIdx.x;
  const int cy = b.lo[1] / 2 + blockIdx.y * BY + threadIdx.y;
  const int cz = (D == 3 ? b.lo[2] / 2 : 0) + blockIdx.z;
  if (cx > b.hi[0] / 2 || cy > b.hi[1] / 2 || (D == 3 && cz > b.hi[2] / 2)) return;
  if (!vm[coincident<D>(gf, b, cx, cy, cz)]) return;
  const long long nc = lin(gc, cx - co.x, cy - co.y, D == 3 ? cz - co.z : 0);
  const int fx = 2 * cx - b.lo[0] + 1, fy = 2 * cy - b.lo[1] + 1, fz = D == 3 ? 2 * cz - b.lo[2] + 1 : 0;
  for (int i = 0; i < ncomp; i++) {
    double s = 0.0;
    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); oz++)
      for (int oy = -1; oy <= 1; oy++)
        for (int ox = -1; ox <= 1; ox++) {
          const double w = (ox ? 0.25 : 0.5) * (oy ? 0.25 : 0.5) * (D == 3 ? (oz ? 0.25 : 0.5) : 1.0);
          s += w * af[i * sf + lin(gf, fx + ox, fy + oy, fz + oz)];
        }
    ac[i * sc + nc] = s;
  }
}

// Bi/trilinear interpolation of a coarse field at the nodes of the fine
// array (of the tiles in act: those holding valid nodes or ghosts).
//   mode 0: dst = interp at every node
//   mode 1: dst = interp at nodes that are not valid
//   mode 2: dst += interp at valid nodes, dst = interp at the others
// dst2 (optional): = interp at nodes that are not valid.
template <int D, typename R>
__global__ __launch_bounds__(256) void k_interp(Geom gc, int3 co, Geom gf, Box b, Mask vm, const int *__restrict__ act,
                                                const R *__restrict__ uc, R *__restrict__ dst, R *__restrict__ dst2,
                                                int mode, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_in(act, gf.m[0], gf.m[1], tx_, ty_, tz_);
  const int x = tx_ * BX + threadIdx.x, y = ty_ * BY + threadIdx.y, z = tz_;
  if (x >= gf.m[0] || y >= gf.m[1]) return;
  const int p[3] = {x, y, z};
  const long long nf = lin(gf, x, y, z);
  const bool ghost = !vm[nf];
  if (mode == 1 && !ghost) return;
  const int cox[3] = {co.x, co.y, co.z};
  int c0[3], c1[3];
  R w1[3];
  for (int a = 0; a < 3; a++) {
    if (a < D) {
      const int I = b.lo[a] - 1 + p[a];       // fine global index (>= 1: boxes keep off the domain boundary)
      c0[a] = I / 2 - cox[a];
      c1[a] = (I & 1) ? c0[a] + 1 : c0[a];
      w1[a] = (I & 1) ? R(0.5) : R(0);
    } else {
      c0[a] = c1[a] = 0;
      w1[a] = R(0);
    }
  }
  for (int i = 0; i < D; i++) {
    R v = R(0);
    for (int sz = 0; sz < (D == 3 ? 2 : 1); sz++)
      for (int sy = 0; sy < 2; sy++)
        for (int sx = 0; sx < 2; sx++) {
          const R w = (sx ? w1[0] : R(1) - w1[0]) * (sy ? w1[1] : R(1) - w1[1]) * (D == 3 ? (sz ? w1[2] : R(1) - w1[2]) : R(1));
          if (w == R(0)) continue;
          v += w * uc[i * gc.N + lin(gc, sx ? c1[0] : c0[0], sy ? c1[1] : c0[1], sz ? c1[2] : c0[2])];
        }
    const long long q = i * gf.N + nf;
    if (mode == 0 || ghost) dst[q] = v;
    else if (mode == 2) dst[q] += v;
    if (dst2 && ghost) dst2[q] = v;
  }
}

// Rows of a refined level's array that are not valid <- v.
template <int D, typename R>
__global__ __launch_bounds__(256) void k_ghost_fill(Geom gf, Mask vm, const int *__restrict__ act, R *__restrict__ a,
                                                    R v, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_in(act, gf.m[0], gf.m[1], tx_, ty_, tz_);
  const int x = tx_ * BX + threadIdx.x, y = ty_ * BY + threadIdx.y, z = tz_;
  if (x >= gf.m[0] || y >= gf.m[1]) return;
  const long long n = lin(gf, x, y, z);
  if (vm[n]) return;
  for (int i = 0; i < D; i++) a[i * gf.N + n] = v;
}

// Restriction of a fine residual onto the covered coarse nodes: full
// weighting over the valid fine nodes only, weights renormalised to sum to
// one where the stencil would reach a node that is not valid (coarse/fine
// boundary).  A covered node's fine node is valid, hence off the array's
// outer ring, so every stencil point lies in the array.
template <int D, typename R>
__global__ __launch_bounds__(256) void k_restrict_cf(Geom gf, Box b, Mask vm, const R *__restrict__ rf, Geom gc,
                                                     int3 co, R *__restrict__ rc, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  const int cx = b.lo[0] / 2 + blockIdx.x * BX + threadIdx.x;
  const int cy = b.lo[1] / 2 + blockIdx.y * BY + threadIdx.y;
  const int cz = (D == 3 ? b.lo[2] / 2 : 0) + blockIdx.z;
  if (cx > b.hi[0] / 2 || cy > b.hi[1] / 2 || (D == 3 && cz > b.hi[2] / 2)) return;
  if (!vm[coincident<D>(gf, b, cx, cy, cz)]) return;
  const long long nc = lin(gc, cx - co.x, cy - co.y, D == 3 ? cz - co.z : 0);
  const int f[3] = {2 * cx - b.lo[0] + 1, 2 * cy - b.lo[1] + 1, D == 3 ? 2 * cz - b.lo[2] + 1 : 0};
  R acc[D], wsum = R(0);
  for (int i = 0; i < D; i++) acc[i] = R(0);
  for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); oz++)
    for (int oy = -1; oy <= 1; oy++)
      for (int ox = -1; ox <= 1; ox++) {
        const long long q = lin(gf, f[0] + ox, f[1] + oy, f[2] + oz);
        if (!vm[q]) continue;
        const R w = (ox ? R(0.25) : R(0.5)) * (oy ? R(0.25) : R(0.5)) * (D == 3 ? (oz ? R(0.25) : R(0.5)) : R(1));
        wsum += w;
        for (int i = 0; i < D; i++) acc[i] += w * rf[i * gf.N + q];
      }
  for (int i = 0; i < D; i++) rc[i * gc.N + nc] = acc[i] / wsum;
}

// Is coarse node (x, y, z) (global) covered by the refined level (b, vm)?
template <int D>
__device__ __forceinline__ bool covered_by(const Geom &gf, const Box &b, Mask vm, int x, int y, int z) {
  if (x < b.lo[0] / 2 || x > b.hi[0] / 2 || y < b.lo[1] / 2 || y > b.hi[1] / 2) return false;
  if (D == 3 && (z < b.lo[2] / 2 || z > b.hi[2] / 2)) return false;
  return vm[coincident<D>(gf, b, x, y, z)] != 0;
}

// Coarse-side effect of a fine correction: the uncovered coarse rows next to
// the level see the correction through the covered (injected) nodes, so
// their residual drops by the coarse operator applied to the injected
// correction.
template <int D, int K, typename R>
struct InjU {
  const R *__restrict__ ef;
  Geom gc, gf;
  int3 co;
  Box b;
  const unsigned char *__restrict__ vm;
  __device__ __forceinline__ R operator()(int k, long long i) const {
    const int x = int(i % gc.m[0]) + co.x, y = int((i / gc.m[0]) % gc.m[1]) + co.y;
    const int z = D == 3 ? int(i / ((long long)gc.m[0] * gc.m[1])) + co.z : 0;
    if (!covered_by<D>(gf, b, vm, x, y, z)) return R(0);
    return ef[k * gf.N + coincident<D>(gf, b, x, y, z)];
  }
};

// One thread per coarse node of the covered bounding box grown by one; only
// uncovered nodes with a row are updated (a node with no covered neighbour
// gets exactly zero).
template <int D, int K, typename R>
__global__ __launch_bounds__(256) void k_cf_update(Geom gc, int3 co, Geom gf, Box b, Mask vm,
                                                   const R *__restrict__ Cc, const R *__restrict__ ef,
                                                   R *__restrict__ rc, const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  const int cx = b.lo[0] / 2 - 1 + blockIdx.x * BX + threadIdx.x;
  const int cy = b.lo[1] / 2 - 1 + blockIdx.y * BY + threadIdx.y;
  const int cz = (D == 3 ? b.lo[2] / 2 - 1 : 0) + blockIdx.z;
  if (cx > b.hi[0] / 2 + 1 || cy > b.hi[1] / 2 + 1 || (D == 3 && cz > b.hi[2] / 2 + 1)) return;
  if (covered_by<D>(gf, b, vm, cx, cy, cz)) return;
  const int p[3] = {cx - co.x, cy - co.y, D == 3 ? cz - co.z : 0};
  const long long n = lin(gc, p[0], p[1], p[2]);
  const int cls = row_class(gc, p);
  if (cls == ROW_DIR) return;
  R acc[D], dg[D];
  rows_at<D, K, R>(gc, Cc, InjU<D, K, R>{ef, gc, gf, co, b, vm}, n, p, cls, acc, dg);
  for (int i = 0; i < D; i++) rc[i * gc.N + n] -= acc[i];
}

// Squared 2-norm partials of r over the composite rows of one level: its
// valid nodes (own_vm; the base grid: non-Dirichlet rows) that the next
// finer level (child_b, child_vm over child_g; none if child_vm is null)
// does not cover.  co: global index of the level's array index 0.
template <int D>
__global__ __launch_bounds__(256) void k_masked_norm(Geom g, const double *__restrict__ r, const unsigned char *own_vm,
                                                     int3 co, Geom child_g, Box child_b,
                                                     const unsigned char *child_vm, double *__restrict__ partial,
                                                     const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  int tx_, ty_, tz_;
  tile_of(tx_, ty_, tz_);
  const int x = tx_ * BX + threadIdx.x, y = ty_ * BY + threadIdx.y, z = tz_;
  double s = 0.0;
  if (x < g.m[0] && y < g.m[1]) {
    const int p[3] = {x, y, z};
    const long long n = lin(g, x, y, z);
    const bool own = own_vm ? own_vm[n] != 0 : row_class(g, p) != ROW_DIR;
    const bool cov = child_vm && covered_by<D>(child_g, child_b, child_vm, x + co.x, y + co.y, z + co.z);
    if (own && !cov)
      for (int i = 0; i < D; i++) {
        const double v = r[i * g.N + n];
        s += v * v;
      }
  }
  block_sum_256(s, partial + block_linear());
}

template <typename R>
__global__ __launch_bounds__(256) void k_axpy(long long n, R *__restrict__ u, const R *__restrict__ e,
                                              const Ctl *__restrict__ ctl) {
  if (skip(ctl)) return;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) u[i] += e[i];
}

}  // namespace emg

// ============================ ragged batching ============================
// Many independent problems of different sizes go through one launch per
// cycle step: the launch grid-strides over a device work list of entries
// (problem, level, operands), each covering a run of tiles.  The per-tile
// bodies are the single-problem ones, so every problem's arithmetic -- and
// its norm partials, indexed by tile -- is the same alone and in a batch.
// Converged problems (their control block says done) are skipped per entry.
namespace emg {

enum {
  BK_JACOBI = 0, BK_JACOBI_NORM = 1, BK_RESID = 2, BK_JZERO = 3, BK_RESTRICT = 4, BK_PROLONG = 5, BK_BOTTOM = 6,
  BK_COPY = 7, BK_ADDC = 8, BK_RESID_F32 = 9, BK_TAIL = 10
};

struct BEnt {
  Geom g, g2;            // level (fine level for restriction / interpolation), coarse level
  const void *C, *a, *b; // moduli, first and second input
  void *out;
  double *partial;
  Ctl *ctl;
  const double *Ainv;
  int nbot, ans;
  int gx, gy, gz;        // tiles of this entry
  long long tile0;       // first global tile
  long long nparts;      // norm partials of the problem (check entries)
  int nzc;               // z-marching entries: chunks per column (tasks = columns x nzc + shell blocks)
  int kind;              // coarse-tail entries: the step (BK_*)
};

struct BList {
  int n, pad;
  long long total;       // tiles over all entries
  BEnt e[1];             // n entries (allocated with capacity)
};

constexpr size_t blist_bytes(int cap) { return sizeof(BList) + sizeof(BEnt) * (cap > 1 ? cap - 1 : 0); }

template <int D, int K, typename R, int KIND>
__global__ __launch_bounds__(256) void k_batch(const BList *__restrict__ L, R omega) {
  const int n = L->n;
  const long long total = L->total;
  for (long long t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L->e[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const BEnt &E = L->e[lo];
    if (E.ctl && E.ctl->done) continue;
    const long long local = t - E.tile0;
    const int tx = int(local % E.gx), ty = int((local / E.gx) % E.gy), tz = int(local / ((long long)E.gx * E.gy));
    if constexpr (KIND == BK_JACOBI || KIND == BK_JACOBI_NORM) {   // stencil entries: gx = split blocks
      body_stencil<D, K, R, MODE_JACOBI, R>(E.g, (const R *)E.C, (const R *)E.a, (const R *)E.b, (R *)E.out, omega,
                                           KIND == BK_JACOBI_NORM ? E.partial + local : nullptr, local);
    } else if constexpr (KIND == BK_RESID) {
      body_stencil<D, K, R, MODE_RESID, R>(E.g, (const R *)E.C, (const R *)E.a, (const R *)E.b, (R *)E.out, R(0),
                                          nullptr, local);
    } else if constexpr (KIND == BK_RESID_F32) {
      body_stencil<D, K, double, MODE_RESID, float>(E.g, (const double *)E.C, (const double *)E.a,
                                                    (const double *)E.b, (float *)E.out, 0.0, E.partial + local,
                                                    local);
    } else if constexpr (KIND == BK_JZERO) {
      body_jacobi_zero<D, K, R>(E.g, (const R *)E.C, (const R *)E.a, (R *)E.out, omega, tx, ty, tz);
    } else if constexpr (KIND == BK_RESTRICT) {
      body_restrict<D, R, R>(E.g, E.g2, (const R *)E.a, (R *)E.out, tx, ty, tz);
    } else if constexpr (KIND == BK_PROLONG) {
      body_prolong<D, R, R>(E.g2, E.g, (const R *)E.a, (R *)E.out, tx, ty, tz);
    } else if constexpr (KIND == BK_BOTTOM) {
      body_bottom<R, R>(E.Ainv, E.nbot, (const R *)E.a, (R *)E.out, (int)local);
    } else {
      const int x = tx * BX + threadIdx.x, y = ty * BY + threadIdx.y, z = tz;
      if (x < E.g.m[0] && y < E.g.m[1]) {
        const long long nn = ((long long)z * E.g.m[1] + y) * E.g.m[0] + x;
        for (int i = 0; i < D; i++) {
          const long long q = i * E.g.N + nn;
          if constexpr (KIND == BK_COPY) ((R *)E.out)[q] = ((const R *)E.a)[q];
          else ((double *)E.out)[q] += double(((const float *)E.a)[q]);
        }
      }
    }
  }
}

// Batched z-marching stencil pass over 3D levels (of one moduli kind) of several
// problems: tasks are the column chunks and shell blocks of each entry
// (k_stencil_zm's workgroups), taken grid-strided by a fixed grid so one
// captured graph serves any batch.  A workgroup finishes a task before it
// takes the next, and no task reads LDS after its last barrier, so tasks
// can reuse the LDS arrays.
template <typename R, int MODE, typename TO, int K = MOD_ANISO>
__global__ __launch_bounds__(256, sizeof(R) == 8 ? 1 : 2) void k_batch_zm(const BList *__restrict__ L, R omega) {
  __shared__ R sC[(K == MOD_ISO ? 9 : 21) * ZM_HP];
  __shared__ R sU[9 * ZM_HP];
  const int n = L->n;
  const long long total = L->total;
  for (long long t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L->e[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const BEnt &E = L->e[lo];
    if (E.ctl && E.ctl->done) continue;
    const long long local = t - E.tile0;
    const Split sp = split_of(E.g);
    const long long nwg = (long long)sp.ntx * sp.nty * E.nzc;
    if (local < nwg) {
      if constexpr (K == MOD_ISO)
        zm_column_iso<R, MODE, TO>(E.g, sp, (const R *)E.C, (const R *)E.a, (const R *)E.b, (TO *)E.out, omega,
                                   E.partial, E.nzc, (unsigned)local, sC, sU);
      else
        zm_column<R, MODE, TO>(E.g, sp, (const R *)E.C, (const R *)E.a, (const R *)E.b, (TO *)E.out, omega,
                               E.partial, E.nzc, (unsigned)local, sC, sU);
    } else {
      body_stencil<3, K, R, MODE, TO>(E.g, (const R *)E.C, (const R *)E.a, (const R *)E.b, (TO *)E.out, omega,
                                      E.partial ? E.partial + (local - nwg) : nullptr, local - nwg);
    }
  }
}

// ---- fused coarse tail ----
// The cycle on a problem's smallest levels (a few hundred nodes each) is one
// launch: a workgroup of TL_WAVES wavefronts walks the problem's list of
// steps -- zero-start sweep, sweeps, residual, restriction, bottom solve,
// interpolation, in the order the per-launch cycle issues them -- with a
// workgroup barrier between steps.  Each wavefront takes 8 x 8 tiles in turn
// (lanes: x = lane % 8, y = lane / 8), which on these levels wastes fewer
// lanes than 64 x 4 tiles; every node is computed by the same per-node body
// as in the separate launches, so the values are bit-identical, and the
// launch and dependent-load latency of each separate kernel (5-10 us, most of
// such a level's time) is paid once.  Entries of a list are grouped by
// problem (tile0 = the problem's index); workgroups take problems
// grid-strided, so a fixed grid serves any batch.
constexpr int TL_X = 8, TL_Y = 8, TL_WAVES = 8, TL_THREADS = 64 * TL_WAVES;

// Rows of e = A^-1 f taken by one wavefront (rows w, w + nw, ...), four at a
// time with all their loads in flight; per row the sum of body_bottom, term
// by term and in its order.
template <typename RI, typename RO>
__device__ __forceinline__ void tail_bottom(const double *__restrict__ Ainv, int n, const RI *__restrict__ f,
                                            RO *__restrict__ e, int w, int nw, int lane) {
  for (int r0 = w; r0 < n; r0 += 4 * nw) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = lane; j < n; j += 64) {
      const double fj = double(f[j]);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int row = r0 + q * nw;
        if (row < n) s[q] += Ainv[(long long)row * n + j] * fj;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int row = r0 + q * nw;
      const double v = wave_sum(s[q]);
      if (lane == 0 && row < n) e[row] = RO(v);
    }
  }
}

template <int D, int K, typename R>
__global__ __launch_bounds__(TL_THREADS) void k_tail(const BList *__restrict__ L, R omega) {
  const int n = L->n;
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int lx = lane % TL_X, ly = lane / TL_X;
  for (long long q = blockIdx.x; q < L->total; q += gridDim.x) {
    int lo = 0, hi = n;   // first entry of problem q
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (L->e[mid].tile0 < q) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= n || (L->e[lo].ctl && L->e[lo].ctl->done)) continue;
    for (int i = lo; i < n && L->e[i].tile0 == q; i++) {
      const BEnt &E = L->e[i];
      const int kind = E.kind;
      if (kind == BK_JACOBI || kind == BK_RESID) {
        const long long nb = split_tiles<TL_X, TL_Y>(E.g).blocks;
        for (long long t = w; t < nb; t += TL_WAVES) {
          if (kind == BK_JACOBI)
            body_stencil<D, K, R, MODE_JACOBI, R, false, TL_X, TL_Y>(E.g, (const R *)E.C, (const R *)E.a,
                                                                   (const R *)E.b, (R *)E.out, omega, nullptr, t,
                                                                   nullptr, lx, ly);
          else
            body_stencil<D, K, R, MODE_RESID, R, false, TL_X, TL_Y>(E.g, (const R *)E.C, (const R *)E.a,
                                                                  (const R *)E.b, (R *)E.out, R(0), nullptr, t,
                                                                  nullptr, lx, ly);
        }
      } else if (kind == BK_BOTTOM) {
        tail_bottom<R, R>(E.Ainv, E.nbot, (const R *)E.a, (R *)E.out, w, TL_WAVES, lane);
      } else {
        // grid tiles of the level written: the level itself (zero-start
        // sweep, interpolation onto it) or the coarse level (restriction)
        const Geom &G = kind == BK_RESTRICT ? E.g2 : E.g;
        const int gx = (G.m[0] + TL_X - 1) / TL_X, gy = (G.m[1] + TL_Y - 1) / TL_Y;
        const long long nt = (long long)gx * gy * G.m[2];
        for (long long t = w; t < nt; t += TL_WAVES) {
          const int tx = int(t % gx), ty = int((t / gx) % gy), tz = int(t / ((long long)gx * gy));
          if (kind == BK_JZERO)
            body_jacobi_zero<D, K, R, TL_X, TL_Y>(E.g, (const R *)E.C, (const R *)E.a, (R *)E.out, omega, tx, ty, tz,
                                                  nullptr, lx, ly);
          else if (kind == BK_RESTRICT)
            body_restrict<D, R, R, TL_X, TL_Y>(E.g, E.g2, (const R *)E.a, (R *)E.out, tx, ty, tz, lx, ly);
          else
            body_prolong<D, R, R, TL_X, TL_Y>(E.g2, E.g, (const R *)E.a, (R *)E.out, tx, ty, tz, lx, ly);
        }
      }
      __syncthreads();   // this step's writes are visible to the whole workgroup
    }
  }
}

__global__ __launch_bounds__(1024) void k_batch_check(const BList *__restrict__ L) {
  for (int i = blockIdx.x; i < L->n; i += gridDim.x) {
    const BEnt &E = L->e[i];
    body_check(E.partial, E.nparts, E.ctl, E.ans);
    __syncthreads();
  }
}

}  // namespace emg
