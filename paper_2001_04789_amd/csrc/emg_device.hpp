// Device-side building blocks of the gfx950 multigrid elasticity solver:
// grid geometry, row classification, the finite-difference rows of the
// operator D_H (product-rule interior rows, traction and Neumann boundary
// rows, Dirichlet rows) and wavefront reductions.
//
// Operator (Sec. 2.1, Sec. 2.1.1 product rule):
//   interior row i:  sum_jkl d_j(C_ijkl) d_l(u_k) + C_ijkl d_jl(u_k)
//   traction row i:  sum over the node's faces of  n_a sum_kl C_iakl dhat_l(u_k)
//   Neumann row i:   sum over the node's Neumann faces of  n_a dhat_a(u_i)
//   Dirichlet row i: u_i
// A node on faces of several kinds takes the Dirichlet row if any of its
// faces is Dirichlet, else the Neumann row if any is Neumann.
// The interior rows are evaluated in "flux form": with e the engineering
// strain of the centre gradient, sum_kl C_ijkl(q) d_l u_k = (C(q) e)_{V(i,j)},
// so the modulus-derivative term is a difference of two neighbour
// stress-like rows and never materialises C_,j.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emg {

enum { BC_DIR = 0, BC_TRAC = 1, BC_PER = 2, BC_NEU = 3 };
enum { ROW_INT = 0, ROW_TRAC = 1, ROW_DIR = 2, ROW_NEU = 3 };
enum { MOD_ISO = 0, MOD_ANISO = 1 };

// Geometry of one level, passed by value to every kernel.
struct Geom {
  int m[3];        // stored nodes per axis (periodic: n-1); m[2] = 1 in 2D
  int dim;
  int per[3];      // periodic flag per axis
  int bc[6];       // face types
  double h[3];     // spacing
  long long N;     // stored nodes
  long long SC;    // component stride of the moduli arrays (>= N, see moduli_stride)
};

// Moduli arrays hold their components at a padded stride: with a stride that
// is a multiple of a large power of two, the 21 component streams a stencil
// reads together fall on the same HBM channels.  Offsetting each component by
// 512 elements spreads them.
__host__ __device__ inline long long moduli_stride(long long N) {
  return N < 4096 ? N : ((N + 511) / 512) * 512 + 512;
}

// Convergence control block living in device memory.  Cycle kernels read
// `done` first and return at once when it is set, so launches queued after
// convergence cost only their launch.
struct Ctl {
  double r0sq;     // squared norm of the first residual (negative until set)
  double rsq;      // squared norm of the latest residual
  double tol2;     // rtol^2
  int done;        // 0 running, 1 converged, 2 diverged (NaN/Inf), 3 cycle cap
  int cycles;      // cycles applied to the iterate being tested
  int ans;         // buffer index holding the answer when done
  int max_cycles;
  int pad[2];
};

template <int D> __host__ __device__ constexpr int nvoigt() { return D == 3 ? 6 : 3; }
template <int D, int K> __host__ __device__ constexpr int nmod() { return K == MOD_ISO ? 2 : (D == 3 ? 21 : 6); }
// Voigt slot of the pair (i,j): 3D 11,22,33,23,31,12 -> 0..5, 2D 11,22,12 -> 0..2
template <int D> __host__ __device__ constexpr int vslot(int i, int j) { return i == j ? i : (D == 2 ? 2 : 6 - i - j); }
// slot of (I,J) in the row-major upper triangle of an n x n symmetric matrix
__host__ __device__ constexpr int utri(int n, int I, int J) {
  return I <= J ? I * n - I * (I - 1) / 2 + (J - I) : J * n - J * (J - 1) / 2 + (I - J);
}

// Full tensor component C_ijkl from the stored constants c[] of one node.
template <int D, int K, typename R>
__device__ __forceinline__ R cfull(const R *c, int i, int j, int k, int l) {
  if constexpr (K == MOD_ISO)
    return c[0] * R((i == j) && (k == l)) + c[1] * (R((i == k) && (j == l)) + R((i == l) && (j == k)));
  else
    return c[utri(nvoigt<D>(), vslot<D>(i, j), vslot<D>(k, l))];
}

// -1 if the node sits on the low end of non-periodic axis a, +1 on the high
// end, 0 otherwise.  Equals the outward normal component of that face.
__device__ __forceinline__ int end_of(const Geom &g, int a, int c) {
  if (g.per[a]) return 0;
  if (c == 0) return -1;
  if (c == g.m[a] - 1) return 1;
  return 0;
}

__device__ __forceinline__ int row_class(const Geom &g, const int p[3]) {
  int on = 0, dir = 0, neu = 0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const int e = a < g.dim ? end_of(g, a, p[a]) : 0;
    if (e) {
      on = 1;
      const int b = g.bc[2 * a + (e > 0)];
      if (b == BC_DIR) dir = 1;
      if (b == BC_NEU) neu = 1;
    }
  }
  return dir ? ROW_DIR : (neu ? ROW_NEU : (on ? ROW_TRAC : ROW_INT));
}

// Normal component of the Neumann face of node p on axis a (0 if p is not
// on a Neumann face of that axis).
__device__ __forceinline__ int neumann_normal(const Geom &g, int a, const int p[3]) {
  const int e = end_of(g, a, p[a]);
  return (e && g.bc[2 * a + (e > 0)] == BC_NEU) ? e : 0;
}

__device__ __forceinline__ long long stride_of(const Geom &g, int a) {
  return a == 0 ? 1LL : (a == 1 ? (long long)g.m[0] : (long long)g.m[0] * g.m[1]);
}

// Linear-index offset of moving by o along axis a from coordinate c
// (periodic axes wrap).
__device__ __forceinline__ long long shift(const Geom &g, int a, int c, int o) {
  int t = c + o;
  if (g.per[a]) {
    if (t < 0) t += g.m[a];
    else if (t >= g.m[a]) t -= g.m[a];
  }
  return (long long)(t - c) * stride_of(g, a);
}

// Accessors for the displacement-like vector the rows act on.
// Element i of the array at `base`.  With a 32-bit unsigned index the byte
// offset is formed in 32 bits (valid while i * sizeof(R) < 2^32), so a load
// from a wavefront-uniform base takes the scalar-base + 32-bit-offset form.
template <typename R, typename I> __device__ __forceinline__ R ld(const R *__restrict__ base, I i) {
  if constexpr (sizeof(I) == 4) return *(const R *)((const char *)base + (unsigned)(i * (unsigned)sizeof(R)));
  else return base[i];
}

template <typename R> struct PtrU {
  const R *__restrict__ p;
  long long N;
  template <typename I> __device__ __forceinline__ R operator()(int k, I i) const { return ld(p + k * N, i); }
};
template <typename R> struct UnitU {   // unit vector e_q
  long long q, N;
  __device__ __forceinline__ R operator()(int k, long long i) const { return (k * N + i == q) ? R(1) : R(0); }
};

// ---- interior rows: product-rule operator with central differences ----
// Loads are issued in two groups (displacement stencil and centre moduli,
// then the neighbour moduli), each complete before its arithmetic starts, so
// a wavefront waits for memory twice per node instead of once per operand.
// N is the component stride of C.  With `f` given, the node's right-hand
// side (f[i NF + n]) is loaded with the first group into fc[], and the centre
// displacement is returned in uc[].  I is the node-index type: long long in
// general, 32-bit unsigned on the interior fast path (offsets then wrap
// modulo 2^32 to the true index).
template <int D, int K, typename R, class U, typename I = long long>
__device__ __forceinline__ void interior_rows(const R *__restrict__ C, long long N, U u, I n, const I om[3],
                                              const I op[3], const R i2h[3], const R ih2[3], R acc[D], R dg[D],
                                              const R *__restrict__ f = nullptr, long long NF = 0, R *fc = nullptr,
                                              R *uc_out = nullptr) {
  constexpr int NP = D == 3 ? 3 : 1;   // mixed pairs (j, l), j < l: (0,1) (0,2) (1,2)
  constexpr int PJ[3] = {0, 0, 1}, PL[3] = {1, 2, 2};
  R uc[D], up[D][D], um[D][D], upp[D][NP], upm[D][NP], ump[D][NP], umm[D][NP];
  if (f) {
#pragma unroll
    for (int k = 0; k < D; k++) fc[k] = ld(f + k * NF, n);
  }
#pragma unroll
  for (int k = 0; k < D; k++) {
    uc[k] = u(k, n);
    if (uc_out) uc_out[k] = uc[k];
#pragma unroll
    for (int j = 0; j < D; j++) {
      up[k][j] = u(k, I(n + op[j]));
      um[k][j] = u(k, I(n + om[j]));
    }
#pragma unroll
    for (int q = 0; q < NP; q++) {
      const int j = PJ[q], l = PL[q];
      upp[k][q] = u(k, I(n + op[j] + op[l]));
      upm[k][q] = u(k, I(n + op[j] + om[l]));
      ump[k][q] = u(k, I(n + om[j] + op[l]));
      umm[k][q] = u(k, I(n + om[j] + om[l]));
    }
  }
  if constexpr (K == MOD_ISO) {
    const R *__restrict__ Cm = C + N;
    R lam = ld(C, n), mu = ld(Cm, n), lp[D], lm[D], mp[D], mm[D];
#pragma unroll
    for (int j = 0; j < D; j++) {
      lp[j] = ld(C, I(n + op[j]));
      lm[j] = ld(C, I(n + om[j]));
      mp[j] = ld(Cm, I(n + op[j]));
      mm[j] = ld(Cm, I(n + om[j]));
    }
    __builtin_amdgcn_sched_barrier(0);
    R G[D][D], H[D][D][D];
#pragma unroll
    for (int k = 0; k < D; k++) {
#pragma unroll
      for (int j = 0; j < D; j++) {
        G[k][j] = (up[k][j] - um[k][j]) * i2h[j];
        H[k][j][j] = (up[k][j] - R(2) * uc[k] + um[k][j]) * ih2[j];
      }
#pragma unroll
      for (int q = 0; q < NP; q++) {
        const int j = PJ[q], l = PL[q];
        R v = ((upp[k][q] - upm[k][q]) - (ump[k][q] - umm[k][q])) * (i2h[j] * i2h[l]);
        H[k][j][l] = v;
        H[k][l][j] = v;
      }
    }
    R divu = R(0);
#pragma unroll
    for (int k = 0; k < D; k++) divu += G[k][k];
#pragma unroll
    for (int i = 0; i < D; i++) {
      R gd = R(0), lap = R(0), s2 = R(0);
#pragma unroll
      for (int k = 0; k < D; k++) gd += H[k][i][k];
#pragma unroll
      for (int j = 0; j < D; j++) {
        lap += H[i][j][j];
        s2 += (j == i ? R(0) : ih2[j]);
      }
      R dlam = (lp[i] - lm[i]) * i2h[i];
      R t1 = dlam * divu;
#pragma unroll
      for (int j = 0; j < D; j++) {
        R dmu = (mp[j] - mm[j]) * i2h[j];
        t1 += dmu * (G[i][j] + G[j][i]);
      }
      acc[i] = (lam + mu) * gd + mu * lap + t1;
      dg[i] = R(-2) * ((lam + R(2) * mu) * ih2[i] + mu * s2);
    }
  } else {
    constexpr int NV = nvoigt<D>(), NC = nmod<D, K>();
    R cc[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) cc[c] = ld(C + c * N, n);
    __builtin_amdgcn_sched_barrier(0);
    R G[D][D], H[D][D][D];
#pragma unroll
    for (int k = 0; k < D; k++) {
#pragma unroll
      for (int j = 0; j < D; j++) {
        G[k][j] = (up[k][j] - um[k][j]) * i2h[j];
        H[k][j][j] = (up[k][j] - R(2) * uc[k] + um[k][j]) * ih2[j];
      }
#pragma unroll
      for (int q = 0; q < NP; q++) {
        const int j = PJ[q], l = PL[q];
        R v = ((upp[k][q] - upm[k][q]) - (ump[k][q] - umm[k][q])) * (i2h[j] * i2h[l]);
        H[k][j][l] = v;
        H[k][l][j] = v;
      }
    }
    R e[NV];
#pragma unroll
    for (int a = 0; a < D; a++) e[a] = G[a][a];
    if constexpr (D == 3) {
      e[3] = G[1][2] + G[2][1];
      e[4] = G[0][2] + G[2][0];
      e[5] = G[0][1] + G[1][0];
    } else {
      e[2] = G[0][1] + G[1][0];
    }
#pragma unroll
    for (int i = 0; i < D; i++) {
      R a2 = R(0), d2 = R(0);
#pragma unroll
      for (int j = 0; j < D; j++) {
#pragma unroll
        for (int k = 0; k < D; k++)
#pragma unroll
          for (int l = 0; l < D; l++) a2 += cc[utri(NV, vslot<D>(i, j), vslot<D>(k, l))] * H[k][j][l];
        d2 += cc[utri(NV, vslot<D>(i, j), vslot<D>(i, j))] * ih2[j];
      }
      acc[i] = a2;
      dg[i] = R(-2) * d2;
    }
    // modulus-derivative term: sum_j [ (C(n+e_j) e)_{V(i,j)} - (C(n-e_j) e)_{V(i,j)} ] / (2 h_j);
    // only the Voigt rows V(i,j) of the neighbours are read (15 of 21 in 3D)
    R cq[D][2][NC];
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
      for (int s = 0; s < 2; s++) {
        const I q = I(n + (s == 0 ? op[j] : om[j]));
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
          for (int J = 0; J < NV; J++) {
            const int c = utri(NV, vslot<D>(i, j), J);
            cq[j][s][c] = ld(C + c * N, q);
          }
      }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
#pragma unroll
      for (int s = 0; s < 2; s++) {
#pragma unroll
        for (int i = 0; i < D; i++) {
          const int Iv = vslot<D>(i, j);
          R sg = R(0);
#pragma unroll
          for (int J = 0; J < NV; J++) sg += cq[j][s][utri(NV, Iv, J)] * e[J];
          acc[i] += (s == 0 ? sg : -sg) * i2h[j];
        }
      }
    }
  }
}

// ---- boundary rows on traction faces (3-point one-sided normal derivatives) ----
template <int D, int K, typename R, class U>
__device__ __forceinline__ void traction_rows(const Geom &g, const R *__restrict__ C, U u, long long n, const int p[3], R acc[D],
                              R dg[D]) {
  constexpr int NC = nmod<D, K>();
  R cc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) cc[c] = C[c * g.SC + n];
  R Gh[D][D], c0[D];
  int en[D];
#pragma unroll
  for (int l = 0; l < D; l++) {
    const R hl = R(g.h[l]);
    en[l] = end_of(g, l, p[l]);
    if (en[l] != 0) {
      const int s = -en[l];   // inward direction
      const long long s1 = shift(g, l, p[l], s), s2 = shift(g, l, p[l], 2 * s);
      c0[l] = R(-3 * s) / (R(2) * hl);
#pragma unroll
      for (int k = 0; k < D; k++)
        Gh[k][l] = R(s) * (R(-3) * u(k, n) + R(4) * u(k, n + s1) - u(k, n + s2)) / (R(2) * hl);
    } else {
      c0[l] = R(0);
      const long long sp = shift(g, l, p[l], 1), sm = shift(g, l, p[l], -1);
#pragma unroll
      for (int k = 0; k < D; k++) Gh[k][l] = (u(k, n + sp) - u(k, n + sm)) / (R(2) * hl);
    }
  }
#pragma unroll
  for (int i = 0; i < D; i++) { acc[i] = R(0); dg[i] = R(0); }
#pragma unroll
  for (int a = 0; a < D; a++) {
    if (en[a] == 0) continue;
    const R na = R(en[a]);
#pragma unroll
    for (int i = 0; i < D; i++) {
      R s = R(0), sd = R(0);
#pragma unroll
      for (int k = 0; k < D; k++)
#pragma unroll
        for (int l = 0; l < D; l++) s += cfull<D, K, R>(cc, i, a, k, l) * Gh[k][l];
#pragma unroll
      for (int l = 0; l < D; l++) sd += cfull<D, K, R>(cc, i, a, i, l) * c0[l];
      acc[i] += na * s;
      dg[i] += na * sd;
    }
  }
}

// ---- boundary rows on Neumann faces: normal derivative of each component ----
template <int D, typename R, class U>
__device__ __forceinline__ void neumann_rows(const Geom &g, U u, long long n, const int p[3], R acc[D], R dg[D]) {
#pragma unroll
  for (int i = 0; i < D; i++) { acc[i] = R(0); dg[i] = R(0); }
#pragma unroll
  for (int a = 0; a < D; a++) {
    const int na = neumann_normal(g, a, p);
    if (!na) continue;
    const R hl = R(g.h[a]);
    const int s = -na;   // inward direction
    const long long s1 = shift(g, a, p[a], s), s2 = shift(g, a, p[a], 2 * s);
    // n_a dhat_a(u) with dhat_a = s (-3 u0 + 4 u1 - u2) / (2h) and n_a s = -1
#pragma unroll
    for (int i = 0; i < D; i++) {
      acc[i] += (R(3) * u(i, n) - R(4) * u(i, n + s1) + u(i, n + s2)) / (R(2) * hl);
      dg[i] += R(3) / (R(2) * hl);
    }
  }
}

// Neighbour offsets (with periodic wrap) of node p for the interior rows.
__device__ __forceinline__ void neighbour_offsets(const Geom &g, const int p[3], long long om[3], long long op[3]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (a < g.dim) {
      om[a] = shift(g, a, p[a], -1);
      op[a] = shift(g, a, p[a], 1);
    } else {
      om[a] = op[a] = 0;
    }
  }
}

// All d rows of D_H at node n (class cls) and their diagonal coefficients.
template <int D, int K, typename R, class U>
__device__ __forceinline__ void rows_at(const Geom &g, const R *__restrict__ C, U u, long long n, const int p[3], int cls,
                                        R acc[D], R dg[D]) {
  if (cls == ROW_INT) {
    long long om[3], op[3];
    neighbour_offsets(g, p, om, op);
    R i2h[3], ih2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      i2h[a] = R(0.5 / g.h[a]);
      ih2[a] = R(1.0 / (g.h[a] * g.h[a]));
    }
    interior_rows<D, K, R, U>(C, g.SC, u, n, om, op, i2h, ih2, acc, dg);
  } else if (cls == ROW_TRAC) {
    traction_rows<D, K, R, U>(g, C, u, n, p, acc, dg);
  } else if (cls == ROW_NEU) {
    neumann_rows<D, R, U>(g, u, n, p, acc, dg);
  } else {
#pragma unroll
    for (int i = 0; i < D; i++) {
      acc[i] = u(i, n);
      dg[i] = R(1);
    }
  }
}

// Diagonal coefficients only (no displacement needed), in precision R from
// moduli stored as RC (each value rounded to R first, so R = float from
// FP64 moduli gives what the FP32 copy of the moduli gives).
template <int D, int K, typename R, typename RC = R>
__device__ __forceinline__ void diag_at(const Geom &g, const RC *__restrict__ C, long long n, const int p[3], int cls,
                                        R dg[D]) {
  if (cls == ROW_DIR) {
#pragma unroll
    for (int i = 0; i < D; i++) dg[i] = R(1);
    return;
  }
  if (cls == ROW_NEU) {
    R s = R(0);
#pragma unroll
    for (int a = 0; a < D; a++)
      if (neumann_normal(g, a, p)) s += R(3) / R(2.0 * g.h[a]);
#pragma unroll
    for (int i = 0; i < D; i++) dg[i] = s;
    return;
  }
  constexpr int NC = nmod<D, K>();
  R cc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) cc[c] = R(C[c * g.SC + n]);
  if (cls == ROW_INT) {
#pragma unroll
    for (int i = 0; i < D; i++) {
      R s = R(0);
#pragma unroll
      for (int j = 0; j < D; j++) s += cfull<D, K, R>(cc, i, j, i, j) * R(1.0 / (g.h[j] * g.h[j]));
      dg[i] = R(-2) * s;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < D; i++) dg[i] = R(0);
#pragma unroll
  for (int a = 0; a < D; a++) {
    int ea = end_of(g, a, p[a]);
    if (!ea) continue;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
      for (int l = 0; l < D; l++) {
        int el = end_of(g, l, p[l]);
        if (!el) continue;
        R c0 = R(3 * el) / R(2.0 * g.h[l]);
        dg[i] += R(ea) * cfull<D, K, R>(cc, i, a, i, l) * c0;
      }
  }
}

// ---- reductions ----
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of v over a 256-thread block, written by thread 0 to *dst.
__device__ __forceinline__ void block_sum_256(double v, double *dst) {
  __shared__ double ws[4];
  const int t = threadIdx.x + threadIdx.y * blockDim.x;
  v = wave_sum(v);
  if ((t & 63) == 0) ws[t >> 6] = v;
  __syncthreads();
  if (t == 0) *dst = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Sum of v over a 128-thread block (two wavefronts), written by thread 0 to *dst.
__device__ __forceinline__ void block_sum_128(double v, double *dst) {
  __shared__ double ws[2];
  const int t = threadIdx.x + threadIdx.y * blockDim.x;
  v = wave_sum(v);
  if ((t & 63) == 0) ws[t >> 6] = v;
  __syncthreads();
  if (t == 0) *dst = ws[0] + ws[1];
}

// Sum of v over a 1024-thread block (16 wavefronts), result to *dst from thread 0.
__device__ __forceinline__ void block_sum_1024(double v, double *dst) {
  __shared__ double ws[16];
  const int t = threadIdx.x;
  v = wave_sum(v);
  if ((t & 63) == 0) ws[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; w++) s += ws[w];
    *dst = s;
  }
}

}  // namespace emg
