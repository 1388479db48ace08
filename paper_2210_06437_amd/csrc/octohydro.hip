// liboctohydro: octree hydro step for gfx950 (AMD Instinct MI355X).
//
// Kernels behind the C-ABI in include/octohydro.h:
//   k_fill   ghost fill into materialised 14^3 tiles (hydro_fill_ghosts)
//   k_step   fused substep: neighbour gather + PPM + Kurganov-Tadmor flux +
//            flux divergence + Runge-Kutta stage combination (hydro_step)
//   k_cfl    global time step: per-cell dx / signal speed, wave64 min, one
//            64-bit atomic min per workgroup (hydro_cfl_dt)
//   k_totals conserved totals with double-double accumulation
//
// The method (paper Sec. IV-C, V-B-1, VI; textbook forms named in the public
// header) is evaluated operation by operation in the order the method states:
// in binary64 every operation is one IEEE-754 operation rounded once, with no
// FMA contraction, so the binary64 path reproduces a plain sequential
// evaluation bit for bit.
//
// Layout in HBM: structure of arrays, field-major: U[f][leaf][z][y][x].
// One 64-lane wavefront owns one leaf in k_step.  For each axis d in turn a
// lane owns one pencil of 8 cells along d (64 pencils per leaf) and streams
// its 14 values (3 ghosts, 8 interior, 3 ghosts) through the PPM recurrences
// in registers; ghost values are read straight from the neighbour leaf in
// global memory (face neighbours only: dimension-by-dimension reconstruction
// never needs edge or corner ghosts).  The per-axis flux differences meet in
// an LDS accumulator, and the last axis finishes the update and writes Uout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "octohydro.h"
#include "octohydro_internal.h"

namespace octohydro {

constexpr int SUB = 8;
constexpr int GH = 3;
constexpr int TW = SUB + 2 * GH;  // 14
constexpr int CELLS = SUB * SUB * SUB;
constexpr int TILE = TW * TW * TW;
constexpr int NF_CORE = 6;  // rho, sx, sy, sz, E, tau
constexpr int ACC_PITCH = 9;  // LDS row pitch (doubles) of the accumulator
constexpr int ACC_PLANE = SUB * ACC_PITCH;
constexpr int ACC_FIELD = SUB * ACC_PLANE;

struct GridArgs {
  int32_t n_leaves;
  int32_t n_nodes;
  int32_t nf;
  int32_t base;
  const int32_t* coord;
  const int32_t* nbr;
  const uint8_t* kind;
  const int32_t* children;
  int32_t* status;
  double gamma;
  double eta1;
};

__device__ __forceinline__ int wrap(int a, int m) {
  a = a < 0 ? a + m : a;
  return a >= m ? a - m : a;
}

// ---------------------------------------------------------------------------
// Ghost values (Sec. VI): same-level copy, injection from a coarser leaf, or
// restriction (mean of the 8 covering cells) from a refined neighbour.
// ---------------------------------------------------------------------------

// Value of the neighbour-side cell with local coordinates l[3] in [0,8) of
// the neighbour block in direction r[3] (each in {-1,0,1}) of `leaf`.
template <typename T>
__device__ __forceinline__ T neighbour_value(const GridArgs& g, const T* __restrict__ Uf, int leaf,
                                             const int (&ic)[3], int blocks, int kind, int id,
                                             const int (&r)[3], const int (&l)[3]) {
  if (kind == HYDRO_SAME_LEAF) {
    return Uf[(size_t)id * CELLS + l[2] * 64 + l[1] * 8 + l[0]];
  }
  if (kind == HYDRO_COARSER_LEAF) {
    int c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int nb = wrap(ic[k] + r[k], blocks);
      c[k] = 4 * (nb & 1) + (l[k] >> 1);
    }
    return Uf[(size_t)id * CELLS + c[2] * 64 + c[1] * 8 + c[0]];
  }
  // refined neighbour: child (l >> 2) on each axis, fine cells (2l + bit) & 7
  const int child = g.children[8 * id + (l[2] >> 2) * 4 + (l[1] >> 2) * 2 + (l[0] >> 2)];
  const T* __restrict__ P = Uf + (size_t)child * CELLS;
  const int fx0 = (2 * l[0]) & 7, fy0 = (2 * l[1]) & 7, fz0 = (2 * l[2]) & 7;
  const T v000 = P[fz0 * 64 + fy0 * 8 + fx0];
  const T v100 = P[fz0 * 64 + fy0 * 8 + fx0 + 1];
  const T v010 = P[fz0 * 64 + (fy0 + 1) * 8 + fx0];
  const T v110 = P[fz0 * 64 + (fy0 + 1) * 8 + fx0 + 1];
  const T v001 = P[(fz0 + 1) * 64 + fy0 * 8 + fx0];
  const T v101 = P[(fz0 + 1) * 64 + fy0 * 8 + fx0 + 1];
  const T v011 = P[(fz0 + 1) * 64 + (fy0 + 1) * 8 + fx0];
  const T v111 = P[(fz0 + 1) * 64 + (fy0 + 1) * 8 + fx0 + 1];
  return T(0.125) * (((v000 + v100) + (v010 + v110)) + ((v001 + v101) + (v011 + v111)));
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_fill(GridArgs g, const T* __restrict__ U, T* __restrict__ G, int64_t total) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx % TILE);
    const int64_t fl = idx / TILE;
    const int leaf = (int)(fl % g.n_leaves);
    const int f = (int)(fl / g.n_leaves);
    const int tp[3] = {t % TW, (t / TW) % TW, t / (TW * TW)};
    int r[3], l[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r[k] = tp[k] < GH ? -1 : (tp[k] >= GH + SUB ? 1 : 0);
      l[k] = tp[k] - GH - SUB * r[k];
    }
    const T* __restrict__ Uf = U + (size_t)f * g.n_leaves * CELLS;
    const int slot = (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
    T v;
    if (slot == 13) {
      v = Uf[(size_t)leaf * CELLS + l[2] * 64 + l[1] * 8 + l[0]];
    } else {
      const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
      const int ic[3] = {c4.y, c4.z, c4.w};
      const int blocks = g.base << c4.x;
      v = neighbour_value<T>(g, Uf, leaf, ic, blocks, g.kind[27 * leaf + slot],
                             g.nbr[27 * leaf + slot], r, l);
    }
    G[idx] = v;
  }
}

// ---------------------------------------------------------------------------
// PPM (Colella & Woodward 1984) as a streaming recurrence along a pencil.
// ---------------------------------------------------------------------------

template <typename T>
struct Ppm {
  T qa, qb;   // q[k-2], q[k-1]
  T qz, qy;   // q[k-3], q[k-4]
  T dmA;      // limited slope of cell k-2
  T qfA;      // interface value between cells k-3 and k-2
  T Rprev;    // right face value of cell k-3
};

// Limited slope of cell j from q[j-1], q[j], q[j+1].
template <typename T>
__device__ __forceinline__ T limited_slope(T qm, T q0, T qp) {
  const T dq = T(0.5) * (qp - qm);
  const T dl = q0 - qm;
  const T dr = qp - q0;
  const T lim = fmin(fabs(dq), fmin(T(2) * fabs(dl), T(2) * fabs(dr)));
  return (dl * dr > T(0)) ? copysign(lim, dq) : T(0);
}

// Monotonised parabola of a cell with centre value c and face values l, r.
template <typename T>
__device__ __forceinline__ void monotonise(T c, T& l, T& r) {
  const T dlr = r - l;
  const T a6 = T(6) * (c - T(0.5) * (l + r));
  const T lo = T(3) * c - T(2) * r;
  const T ro = T(3) * c - T(2) * l;
  const bool flat = (r - c) * (c - l) <= T(0);
  const bool fix_l = dlr * a6 > dlr * dlr;
  const bool fix_r = -(dlr * dlr) > dlr * a6;
  const T nl = flat ? c : (fix_l ? lo : l);
  const T nr = flat ? c : (fix_l ? r : (fix_r ? ro : r));
  l = nl;
  r = nr;
}

// Feed q[k]; when k >= 5, returns the face states of the face between tile
// cells k-3 and k-2 in (UL, UR).  k is a compile-time constant after unroll.
template <typename T>
__device__ __forceinline__ void ppm_push(Ppm<T>& s, T qn, int k, T& UL, T& UR) {
  T dm_new = T(0), qf_new = T(0), Lc = T(0), Rc = T(0);
  if (k >= 2) dm_new = limited_slope(s.qa, s.qb, qn);
  if (k >= 3) qf_new = T(0.5) * (s.qa + s.qb) - (dm_new - s.dmA) * T(1.0 / 6.0);
  if (k >= 4) {
    Lc = s.qfA;
    Rc = qf_new;
    monotonise(s.qa, Lc, Rc);
  }
  if (k >= 5) {
    UL = s.Rprev;
    UR = Lc;
  }
  s.Rprev = Rc;
  s.qfA = qf_new;
  s.dmA = dm_new;
  s.qy = s.qz;
  s.qz = s.qa;
  s.qa = s.qb;
  s.qb = qn;
}

// ---------------------------------------------------------------------------
// EOS and Kurganov-Tadmor flux
// ---------------------------------------------------------------------------

template <typename T>
struct Phys {
  T gamma, gm1, eta1;
};

// rinv = 1/rho, p, c for conserved state (rho, sx, sy, sz, E, tau).
template <typename T>
__device__ __forceinline__ bool eos(const Phys<T>& ph, T rho, T sx, T sy, T sz, T E, T tau,
                                    T& rinv, T& p, T& c) {
  rinv = T(1) / rho;
  const T ss = (sx * sx + sy * sy) + sz * sz;
  T ei = E - T(0.5) * ss * rinv;
  if (ei < ph.eta1 * E) ei = pow(tau, ph.gamma);
  p = ph.gm1 * ei;
  c = sqrt(ph.gamma * p * rinv);
  return !(rho > T(0)) || !(p > T(0));
}

// ---------------------------------------------------------------------------
// Fused substep kernel
// ---------------------------------------------------------------------------

struct StepArgs {
  GridArgs g;
  const void* U0;
  const void* Uk;
  void* Uout;
  const double* dt;
  double beta;
  int32_t leaf_base;  // first leaf (per-leaf launches); 0 for the batch
  int32_t remap;      // 1: spread contiguous leaf ranges over the 8 XCDs
};

// Strides of a cell (pos along axis D, a, b transverse) inside a leaf.
template <int D>
struct Axes;
template <>
struct Axes<0> {
  static constexpr int SD = 1, SA = 8, SB = 64, A = 1, B = 2;
};
template <>
struct Axes<1> {
  static constexpr int SD = 8, SA = 1, SB = 64, A = 0, B = 2;
};
template <>
struct Axes<2> {
  static constexpr int SD = 64, SA = 1, SB = 8, A = 0, B = 1;
};

template <int D>
__device__ __forceinline__ int acc_index(int i, int a, int b) {
  int c[3];
  c[D] = i;
  c[Axes<D>::A] = a;
  c[Axes<D>::B] = b;
  return c[2] * ACC_PLANE + c[1] * ACC_PITCH + c[0];
}

struct LeafInfo {
  int leaf;
  int ic[3];
  int blocks;
  int kind_lo[3], id_lo[3], kind_hi[3], id_hi[3];
};

// Value at tile position k (0..13) of the pencil along D through (a, b).
template <typename T, int D>
__device__ __forceinline__ T pencil_value(const GridArgs& g, const T* __restrict__ Uf,
                                          const LeafInfo& li, int k, int a, int b) {
  using X = Axes<D>;
  if (k >= GH && k < GH + SUB)
    return Uf[(size_t)li.leaf * CELLS + (k - GH) * X::SD + a * X::SA + b * X::SB];
  const bool hi = k >= GH + SUB;
  int r[3] = {0, 0, 0}, l[3];
  r[D] = hi ? 1 : -1;
  l[D] = hi ? k - GH - SUB : k - GH + SUB;
  l[X::A] = a;
  l[X::B] = b;
  return neighbour_value<T>(g, Uf, li.leaf, li.ic, li.blocks, hi ? li.kind_hi[D] : li.kind_lo[D],
                            hi ? li.id_hi[D] : li.id_lo[D], r, l);
}

// One axis of the substep for one leaf; lane = pencil (a, b).
template <typename T, int NF, int D>
__device__ __forceinline__ void axis_pass(const StepArgs& s, const Phys<T>& ph, const LeafInfo& li,
                                          double* __restrict__ acc, double dt, double inv_dx,
                                          int lane, bool& bad) {
  const GridArgs& g = s.g;
  const int a = lane & 7, b = lane >> 3;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const T* __restrict__ Uk = static_cast<const T*>(s.Uk);

  // Face speeds from the core pass, reused by the passive species.
  T vLf[SUB + 1], vRf[SUB + 1], haf[SUB + 1];

  // ---- core fields: rho, s, E, tau ----
  {
    Ppm<T> st[NF_CORE];
    double Hprev[NF_CORE];
    T UL[NF_CORE], UR[NF_CORE];
#pragma unroll
    for (int f = 0; f < NF_CORE; ++f) {
      st[f] = Ppm<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
      Hprev[f] = 0.0;
      UL[f] = UR[f] = T(0);
    }
#pragma unroll
    for (int k = 0; k < TW; ++k) {
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        const T q = pencil_value<T, D>(g, Uk + f * fs, li, k, a, b);
        ppm_push(st[f], q, k, UL[f], UR[f]);
      }
      if (k >= 5) {
        const int face = k - 5;  // low face of interior cell `face`
        T riL, pL, cL, riR, pR, cR;
        bad |= eos(ph, UL[0], UL[1], UL[2], UL[3], UL[4], UL[5], riL, pL, cL);
        bad |= eos(ph, UR[0], UR[1], UR[2], UR[3], UR[4], UR[5], riR, pR, cR);
        const T vL = UL[1 + D] * riL;
        const T vR = UR[1 + D] * riR;
        const T ha = T(0.5) * fmax(fabs(vL) + cL, fabs(vR) + cR);
        vLf[face] = vL;
        vRf[face] = vR;
        haf[face] = ha;
        T FL[NF_CORE], FR[NF_CORE];
        FL[0] = UL[1 + D];
        FR[0] = UR[1 + D];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          FL[1 + m] = UL[1 + m] * vL;
          FR[1 + m] = UR[1 + m] * vR;
        }
        FL[1 + D] = FL[1 + D] + pL;
        FR[1 + D] = FR[1 + D] + pR;
        FL[4] = (UL[4] + pL) * vL;
        FR[4] = (UR[4] + pR) * vR;
        FL[5] = UL[5] * vL;
        FR[5] = UR[5] * vR;
#pragma unroll
        for (int f = 0; f < NF_CORE; ++f) {
          const T Ht = T(0.5) * (FL[f] + FR[f]) - ha * (UR[f] - UL[f]);
          const double H = (double)Ht;
          if (face >= 1) {
            const int i = face - 1;
            const double dH = H - Hprev[f];
            const int ai = f * ACC_FIELD + acc_index<D>(i, a, b);
            if constexpr (D == 0) {
              acc[ai] = dH;
            } else if constexpr (D == 1) {
              acc[ai] = acc[ai] + dH;
            } else {
              const double sum = acc[ai] + dH;
              const double lrate = -sum * inv_dx;
              const int cell = (i)*64 + b * 8 + a;
              const size_t at = (size_t)f * fs + (size_t)li.leaf * CELLS + cell;
              const double t = (double)st[f].qy + dt * lrate;
              double out;
              if (s.U0) {
                const double u0 = (double)static_cast<const T*>(s.U0)[at];
                out = u0 + s.beta * (t - u0);
              } else {
                out = t;
              }
              static_cast<T*>(s.Uout)[at] = (T)out;
            }
          }
          Hprev[f] = H;
        }
      }
    }
  }

  // ---- passive species: flux rho_k v_n with the same dissipation ----
#pragma unroll 1
  for (int f = NF_CORE; f < NF; ++f) {
    Ppm<T> st{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    double Hprev = 0.0;
    T ULs = T(0), URs = T(0);
#pragma unroll
    for (int k = 0; k < TW; ++k) {
      const T q = pencil_value<T, D>(g, Uk + f * fs, li, k, a, b);
      ppm_push(st, q, k, ULs, URs);
      if (k >= 5) {
        const int face = k - 5;
        const T Ht = T(0.5) * (ULs * vLf[face] + URs * vRf[face]) - haf[face] * (URs - ULs);
        const double H = (double)Ht;
        if (face >= 1) {
          const int i = face - 1;
          const double dH = H - Hprev;
          const int ai = f * ACC_FIELD + acc_index<D>(i, a, b);
          if constexpr (D == 0) {
            acc[ai] = dH;
          } else if constexpr (D == 1) {
            acc[ai] = acc[ai] + dH;
          } else {
            const double sum = acc[ai] + dH;
            const double lrate = -sum * inv_dx;
            const int cell = i * 64 + b * 8 + a;
            const size_t at = (size_t)f * fs + (size_t)li.leaf * CELLS + cell;
            const double t = (double)st.qy + dt * lrate;
            double out;
            if (s.U0) {
              const double u0 = (double)static_cast<const T*>(s.U0)[at];
              out = u0 + s.beta * (t - u0);
            } else {
              out = t;
            }
            static_cast<T*>(s.Uout)[at] = (T)out;
          }
        }
        Hprev = H;
      }
    }
  }
}

template <typename T, int NF>
__global__ void __launch_bounds__(64) k_step(StepArgs s) {
  __shared__ double acc[NF * ACC_FIELD];
  const GridArgs& g = s.g;
  int bid = blockIdx.x;
  if (s.remap) {
    // contiguous (Morton-ordered) leaf ranges per XCD: blocks are dealt to
    // the 8 XCDs round-robin, so block b runs on XCD b % 8
    const int n = g.n_leaves, q = n >> 3, r = n & 7;
    const int xcd = bid & 7, j = bid >> 3;
    bid = xcd * q + min(xcd, r) + j;
  }
  const int leaf = s.leaf_base + bid;
  if (leaf >= g.n_leaves) return;
  const int lane = threadIdx.x;

  LeafInfo li;
  li.leaf = leaf;
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  li.ic[0] = c4.y;
  li.ic[1] = c4.z;
  li.ic[2] = c4.w;
  li.blocks = g.base << c4.x;
  // face-neighbour slots: -x 12, +x 14, -y 10, +y 16, -z 4, +z 22
  const int slo[3] = {12, 10, 4}, shi[3] = {14, 16, 22};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    li.kind_lo[d] = g.kind[27 * leaf + slo[d]];
    li.id_lo[d] = g.nbr[27 * leaf + slo[d]];
    li.kind_hi[d] = g.kind[27 * leaf + shi[d]];
    li.id_hi[d] = g.nbr[27 * leaf + shi[d]];
  }
  const double dt = *s.dt;
  const double inv_dx = (double)(SUB * li.blocks);
  Phys<T> ph;
  ph.gamma = (T)g.gamma;
  ph.gm1 = (T)(g.gamma - 1.0);
  ph.eta1 = (T)g.eta1;

  bool bad = false;
  axis_pass<T, NF, 0>(s, ph, li, acc, dt, inv_dx, lane, bad);
  __syncthreads();
  axis_pass<T, NF, 1>(s, ph, li, acc, dt, inv_dx, lane, bad);
  __syncthreads();
  axis_pass<T, NF, 2>(s, ph, li, acc, dt, inv_dx, lane, bad);
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
}

// ---------------------------------------------------------------------------
// CFL time step
// ---------------------------------------------------------------------------

__global__ void k_dt_init(double* dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    *reinterpret_cast<unsigned long long*>(dt) = 0x7FF0000000000000ull;  // +inf
}

__global__ void k_dt_final(double* dt, double cfl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dt = cfl * *dt;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cfl(GridArgs g, const T* __restrict__ U, double* dt) {
  __shared__ double part[4];
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const double gm1 = g.gamma - 1.0;
  double best = INFINITY;
  for (int leaf = blockIdx.x; leaf < g.n_leaves; leaf += gridDim.x) {
    const int L = g.coord[4 * leaf];
    const double dx = 1.0 / (double)(SUB * (g.base << L));
    for (int cell = threadIdx.x; cell < CELLS; cell += blockDim.x) {
      const size_t at = (size_t)leaf * CELLS + cell;
      const double rho = (double)U[at], sx = (double)U[fs + at], sy = (double)U[2 * fs + at];
      const double sz = (double)U[3 * fs + at], E = (double)U[4 * fs + at];
      const double rinv = 1.0 / rho;
      const double ss = (sx * sx + sy * sy) + sz * sz;
      double ei = E - 0.5 * ss * rinv;
      if (ei < g.eta1 * E) ei = pow((double)U[5 * fs + at], g.gamma);
      const double p = gm1 * ei;
      const double c = sqrt(g.gamma * p * rinv);
      const double vmax = fmax(fmax(fabs(sx * rinv), fabs(sy * rinv)), fabs(sz * rinv));
      const double q = dx / (vmax + c);
      best = fmin(best, q);
    }
  }
  best = wave_min(best);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[w] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmin(m, part[i]);
    // positive doubles order like their bit patterns
    atomicMin(reinterpret_cast<unsigned long long*>(dt), (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
// Conserved totals (double-double accumulation, fixed reduction order)
// ---------------------------------------------------------------------------

struct DD {
  double hi, lo;
};

__device__ __forceinline__ DD dd_add(DD a, DD b) {
  const double s = a.hi + b.hi;
  const double bb = s - a.hi;
  const double e = (a.hi - (s - bb)) + (b.hi - bb);
  const double lo = e + (a.lo + b.lo);
  const double hi = s + lo;
  return DD{hi, lo - (hi - s)};
}

constexpr int TOT_BLOCKS = 1024;
constexpr int TOT_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(TOT_THREADS)
    k_totals(GridArgs g, const T* __restrict__ U, double* __restrict__ partial) {
  __shared__ DD red[TOT_THREADS];
  const size_t fs = (size_t)g.n_leaves * CELLS;
  for (int f = 0; f < g.nf; ++f) {
    DD acc{0.0, 0.0};
    for (int leaf = blockIdx.x; leaf < g.n_leaves; leaf += gridDim.x) {
      const int L = g.coord[4 * leaf];
      const double dx = 1.0 / (double)(SUB * (g.base << L));
      const double dv = dx * dx * dx;
      for (int cell = threadIdx.x; cell < CELLS; cell += TOT_THREADS)
        acc = dd_add(acc, DD{(double)U[(size_t)f * fs + (size_t)leaf * CELLS + cell] * dv, 0.0});
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = TOT_THREADS / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] = dd_add(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partial[2 * ((size_t)f * gridDim.x + blockIdx.x)] = red[0].hi;
      partial[2 * ((size_t)f * gridDim.x + blockIdx.x) + 1] = red[0].lo;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(TOT_THREADS)
    k_totals_final(const double* __restrict__ partial, int nblocks, int nf, double* out) {
  __shared__ DD red[TOT_THREADS];
  for (int f = 0; f < nf; ++f) {
    DD acc{0.0, 0.0};
    for (int i = threadIdx.x; i < nblocks; i += TOT_THREADS)
      acc = dd_add(acc, DD{partial[2 * ((size_t)f * nblocks + i)],
                           partial[2 * ((size_t)f * nblocks + i) + 1]});
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = TOT_THREADS / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] = dd_add(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[f] = red[0].hi + red[0].lo;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Table validation (HYDRO_FLAG_VALIDATE)
// ---------------------------------------------------------------------------

__global__ void k_validate(GridArgs g) {
  const int64_t total = (int64_t)g.n_leaves * 27;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kd = g.kind[i];
    const int id = g.nbr[i];
    bool ok = kd == HYDRO_SAME_LEAF || kd == HYDRO_COARSER_LEAF || kd == HYDRO_SAME_REFINED;
    if (kd == HYDRO_SAME_REFINED) {
      ok = ok && id >= 0 && id < g.n_nodes;
      if (ok)
        for (int c = 0; c < 8; ++c) {
          const int ch = g.children[8 * id + c];
          ok = ok && ch >= -1 && ch < g.n_leaves;
        }
    } else {
      ok = ok && id >= 0 && id < g.n_leaves;
    }
    if (!ok) atomicOr(g.status, (int)HYDRO_STATUS_TABLE);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(HYDRO_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

static int check_grid(const hydro_grid* gr, const char* fn) {
  if (!gr) return fail(HYDRO_E_ARG, "%s: grid is NULL", fn);
  if (gr->n_leaves <= 0) return fail(HYDRO_E_ARG, "%s: n_leaves must be positive", fn);
  if (gr->n_fields < NF_CORE || gr->n_fields > 16)
    return fail(HYDRO_E_ARG, "%s: n_fields must be in [6,16], got %d", fn, gr->n_fields);
  if (gr->dtype != HYDRO_F64 && gr->dtype != HYDRO_F32)
    return fail(HYDRO_E_ARG, "%s: unknown dtype %d", fn, gr->dtype);
  if (gr->base <= 0) return fail(HYDRO_E_ARG, "%s: base must be positive", fn);
  if (!gr->leaf_coord_dev || !gr->nbr_dev || !gr->nbr_kind_dev)
    return fail(HYDRO_E_ARG, "%s: table pointers must be set", fn);
  if (gr->n_nodes > 0 && !gr->children_dev)
    return fail(HYDRO_E_ARG, "%s: children_dev is NULL but n_nodes > 0", fn);
  if (!(gr->gamma > 1.0)) return fail(HYDRO_E_ARG, "%s: gamma must exceed 1", fn);
  return HYDRO_OK;
}

static GridArgs grid_args(const hydro_grid* gr) {
  GridArgs g;
  g.n_leaves = gr->n_leaves;
  g.n_nodes = gr->n_nodes;
  g.nf = gr->n_fields;
  g.base = gr->base;
  g.coord = gr->leaf_coord_dev;
  g.nbr = gr->nbr_dev;
  g.kind = gr->nbr_kind_dev;
  g.children = gr->children_dev;
  g.status = gr->status_dev;
  g.gamma = gr->gamma;
  g.eta1 = gr->dual_energy_eta1;
  return g;
}

static int grid_blocks(int64_t work, int threads, int cap) {
  int64_t b = (work + threads - 1) / threads;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

template <typename T, int NF>
static hipError_t launch_step_nf(const StepArgs& a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_step<T, NF>), dim3(blocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_step_t(const StepArgs& a, int blocks, hipStream_t st) {
  switch (a.g.nf) {
    case 6: return launch_step_nf<T, 6>(a, blocks, st);
    case 7: return launch_step_nf<T, 7>(a, blocks, st);
    case 8: return launch_step_nf<T, 8>(a, blocks, st);
    case 9: return launch_step_nf<T, 9>(a, blocks, st);
    case 10: return launch_step_nf<T, 10>(a, blocks, st);
    case 11: return launch_step_nf<T, 11>(a, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t launch_step(const StepArgs& a, int dtype, int blocks, hipStream_t st) {
  return dtype == HYDRO_F64 ? launch_step_t<double>(a, blocks, st)
                            : launch_step_t<float>(a, blocks, st);
}

static int validate_table(const hydro_grid* gr, hipStream_t st) {
  if (!gr->status_dev)
    return fail(HYDRO_E_ARG, "HYDRO_FLAG_VALIDATE needs grid->status_dev");
  GridArgs g = grid_args(gr);
  hipLaunchKernelGGL(k_validate, dim3(grid_blocks((int64_t)g.n_leaves * 27, 256, 4096)),
                     dim3(256), 0, st, g);
  HIP_TRY(hipGetLastError());
  int32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, gr->status_dev, sizeof(flag), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (flag & HYDRO_STATUS_TABLE) return fail(HYDRO_E_TABLE, "neighbour table failed validation");
  return HYDRO_OK;
}

static int step_common(const hydro_grid* gr, const void* U0, const void* Uk, void* Uout,
                       const double* dt, double beta, uint32_t flags, const char* fn,
                       StepArgs& a) {
  int rc = check_grid(gr, fn);
  if (rc) return rc;
  if (gr->n_fields > 11)
    return fail(HYDRO_E_UNSUPPORTED, "%s: n_fields %d > 11 not built", fn, gr->n_fields);
  if (!Uk || !Uout || !dt) return fail(HYDRO_E_ARG, "%s: Uk, Uout and dt must be set", fn);
  if (Uout == Uk || (U0 && Uout == U0))
    return fail(HYDRO_E_ARG, "%s: Uout may not alias an input", fn);
  if (flags & ~HYDRO_FLAG_VALIDATE) return fail(HYDRO_E_ARG, "%s: unknown flags", fn);
  a.g = grid_args(gr);
  a.U0 = U0;
  a.Uk = Uk;
  a.Uout = Uout;
  a.dt = dt;
  a.beta = beta;
  a.leaf_base = 0;
  a.remap = 1;
  return HYDRO_OK;
}

static int cfl_launch(const hydro_grid* gr, const void* U, double cfl, double* dt, hipStream_t st) {
  GridArgs g = grid_args(gr);
  hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, st, dt);
  HIP_TRY(hipGetLastError());
  const int blocks = grid_blocks(g.n_leaves, 1, 4096);
  if (gr->dtype == HYDRO_F64)
    hipLaunchKernelGGL(k_cfl<double>, dim3(blocks), dim3(256), 0, st, g,
                       static_cast<const double*>(U), dt);
  else
    hipLaunchKernelGGL(k_cfl<float>, dim3(blocks), dim3(256), 0, st, g,
                       static_cast<const float*>(U), dt);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(64), 0, st, dt, cfl);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

static int rk3_launch(const hydro_grid* gr, const void* Un, void* W1, void* W2, void* Unext,
                      double cfl, double* dt, hipStream_t st) {
  int rc = check_grid(gr, "hydro_rk3_step");
  if (rc) return rc;
  if (!Un || !W1 || !W2 || !Unext || !dt)
    return fail(HYDRO_E_ARG, "hydro_rk3_step: null buffer");
  if (Unext == Un || Unext == W2 || W1 == W2 || W1 == Un || W2 == Un)
    return fail(HYDRO_E_ARG, "hydro_rk3_step: buffers alias");
  if (cfl > 0.0) {
    rc = cfl_launch(gr, Un, cfl, dt, st);
    if (rc) return rc;
  }
  StepArgs a;
  rc = step_common(gr, nullptr, Un, W1, dt, 1.0, 0, "hydro_rk3_step", a);
  if (rc) return rc;
  HIP_TRY(launch_step(a, gr->dtype, gr->n_leaves, st));
  a.U0 = Un;
  a.Uk = W1;
  a.Uout = W2;
  a.beta = 0.25;
  HIP_TRY(launch_step(a, gr->dtype, gr->n_leaves, st));
  a.Uk = W2;
  a.Uout = Unext;
  a.beta = 2.0 / 3.0;
  HIP_TRY(launch_step(a, gr->dtype, gr->n_leaves, st));
  return HYDRO_OK;
}

// library-owned scratch (per device), grown on demand
struct Scratch {
  std::mutex mu;
  std::vector<void*> ptr;
  std::vector<size_t> size;
};
static Scratch g_scratch;

static int scratch_get(size_t bytes, void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch.mu);
  if ((int)g_scratch.ptr.size() <= dev) {
    g_scratch.ptr.resize(dev + 1, nullptr);
    g_scratch.size.resize(dev + 1, 0);
  }
  if (g_scratch.size[dev] < bytes) {
    if (g_scratch.ptr[dev]) HIP_TRY(hipFree(g_scratch.ptr[dev]));
    g_scratch.ptr[dev] = nullptr;
    g_scratch.size[dev] = 0;
    HIP_TRY(hipMalloc(&g_scratch.ptr[dev], bytes));
    g_scratch.size[dev] = bytes;
  }
  *out = g_scratch.ptr[dev];
  return HYDRO_OK;
}

// stream pool for the per-leaf launch mode (default priority)
struct StreamPool {
  std::mutex mu;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  int device = -1;
};
static StreamPool g_pool;

struct Graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace octohydro

using namespace octohydro;

extern "C" {

int hydro_version(void) { return 100; }

const char* hydro_last_error(void) { return error_buffer(); }

int hydro_fill_ghosts(const hydro_grid* gr, const void* U, void* G, void* stream) {
  clear_error();
  int rc = check_grid(gr, "hydro_fill_ghosts");
  if (rc) return rc;
  if (!U || !G) return fail(HYDRO_E_ARG, "hydro_fill_ghosts: U and G must be set");
  if (U == G) return fail(HYDRO_E_ARG, "hydro_fill_ghosts: G may not alias U");
  hipStream_t st = static_cast<hipStream_t>(stream);
  GridArgs g = grid_args(gr);
  const int64_t total = (int64_t)g.nf * g.n_leaves * TILE;
  const int blocks = grid_blocks(total, 256, 1 << 16);
  if (gr->dtype == HYDRO_F64)
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, st, g,
                       static_cast<const double*>(U), static_cast<double*>(G), total);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(256), 0, st, g,
                       static_cast<const float*>(U), static_cast<float*>(G), total);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int hydro_step(const hydro_grid* gr, const void* U0, const void* Uk, void* Uout, const double* dt,
               double beta, uint32_t flags, void* stream) {
  clear_error();
  StepArgs a;
  int rc = step_common(gr, U0, Uk, Uout, dt, beta, flags, "hydro_step", a);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (flags & HYDRO_FLAG_VALIDATE) {
    rc = validate_table(gr, st);
    if (rc) return rc;
  }
  HIP_TRY(launch_step(a, gr->dtype, gr->n_leaves, st));
  return HYDRO_OK;
}

int hydro_step_per_leaf(const hydro_grid* gr, const void* U0, const void* Uk, void* Uout,
                        const double* dt, double beta, int32_t n_streams, void* stream) {
  clear_error();
  StepArgs a;
  int rc = step_common(gr, U0, Uk, Uout, dt, beta, 0, "hydro_step_per_leaf", a);
  if (rc) return rc;
  if (n_streams < 1 || n_streams > 1024)
    return fail(HYDRO_E_ARG, "hydro_step_per_leaf: n_streams must be in [1,1024]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool.mu);
  if (g_pool.device != dev) {
    for (auto s : g_pool.streams) (void)hipStreamDestroy(s);
    for (auto e : g_pool.events) (void)hipEventDestroy(e);
    g_pool.streams.clear();
    g_pool.events.clear();
    g_pool.device = dev;
  }
  while ((int)g_pool.streams.size() < n_streams) {
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    g_pool.streams.push_back(s);
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    g_pool.events.push_back(e);
  }
  // pool streams start after the work already queued on `stream`
  HIP_TRY(hipEventRecord(g_pool.events[0], st));
  for (int i = 0; i < n_streams; ++i) HIP_TRY(hipStreamWaitEvent(g_pool.streams[i], g_pool.events[0], 0));
  a.remap = 0;
  for (int leaf = 0; leaf < gr->n_leaves; ++leaf) {
    a.leaf_base = leaf;
    HIP_TRY(launch_step(a, gr->dtype, 1, g_pool.streams[leaf % n_streams]));
  }
  for (int i = 0; i < n_streams; ++i) {
    HIP_TRY(hipEventRecord(g_pool.events[i], g_pool.streams[i]));
    HIP_TRY(hipStreamWaitEvent(st, g_pool.events[i], 0));
  }
  return HYDRO_OK;
}

int hydro_cfl_dt(const hydro_grid* gr, const void* U, double cfl, double* dt, void* stream) {
  clear_error();
  int rc = check_grid(gr, "hydro_cfl_dt");
  if (rc) return rc;
  if (!U || !dt) return fail(HYDRO_E_ARG, "hydro_cfl_dt: U and dt must be set");
  if (!(cfl > 0.0)) return fail(HYDRO_E_ARG, "hydro_cfl_dt: cfl must be positive");
  return cfl_launch(gr, U, cfl, dt, static_cast<hipStream_t>(stream));
}

int hydro_totals(const hydro_grid* gr, const void* U, double* totals, void* stream) {
  clear_error();
  int rc = check_grid(gr, "hydro_totals");
  if (rc) return rc;
  if (!U || !totals) return fail(HYDRO_E_ARG, "hydro_totals: U and totals must be set");
  hipStream_t st = static_cast<hipStream_t>(stream);
  GridArgs g = grid_args(gr);
  const int blocks = grid_blocks(g.n_leaves, 1, TOT_BLOCKS);
  void* part = nullptr;
  rc = scratch_get(sizeof(double) * 2 * (size_t)blocks * g.nf, &part);
  if (rc) return rc;
  if (gr->dtype == HYDRO_F64)
    hipLaunchKernelGGL(k_totals<double>, dim3(blocks), dim3(TOT_THREADS), 0, st, g,
                       static_cast<const double*>(U), static_cast<double*>(part));
  else
    hipLaunchKernelGGL(k_totals<float>, dim3(blocks), dim3(TOT_THREADS), 0, st, g,
                       static_cast<const float*>(U), static_cast<double*>(part));
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(TOT_THREADS), 0, st,
                     static_cast<const double*>(part), blocks, g.nf, totals);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int hydro_rk3_step(const hydro_grid* gr, const void* Un, void* W1, void* W2, void* Unext,
                   double cfl, double* dt, void* stream) {
  clear_error();
  return rk3_launch(gr, Un, W1, W2, Unext, cfl, dt, static_cast<hipStream_t>(stream));
}

int hydro_rk3_graph_create(const hydro_grid* gr, const void* Un, void* W1, void* W2,
                           void* Unext, double cfl, double* dt, void** graph_out) {
  clear_error();
  if (!graph_out) return fail(HYDRO_E_ARG, "hydro_rk3_graph_create: graph_out is NULL");
  *graph_out = nullptr;
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(HYDRO_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  int rc = rk3_launch(gr, Un, W1, W2, Unext, cfl, dt, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(HYDRO_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(HYDRO_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  Graph* h = new Graph;
  h->graph = graph;
  h->exec = exec;
  *graph_out = h;
  return HYDRO_OK;
}

int hydro_graph_launch(void* graph, void* stream) {
  clear_error();
  if (!graph) return fail(HYDRO_E_ARG, "hydro_graph_launch: graph is NULL");
  Graph* h = static_cast<Graph*>(graph);
  HIP_TRY(hipGraphLaunch(h->exec, static_cast<hipStream_t>(stream)));
  return HYDRO_OK;
}

int hydro_graph_destroy(void* graph) {
  clear_error();
  if (!graph) return HYDRO_OK;
  Graph* h = static_cast<Graph*>(graph);
  if (h->exec) HIP_TRY(hipGraphExecDestroy(h->exec));
  if (h->graph) HIP_TRY(hipGraphDestroy(h->graph));
  delete h;
  return HYDRO_OK;
}

int hydro_check_status(const hydro_grid* gr, void* stream) {
  clear_error();
  if (!gr || !gr->status_dev) return fail(HYDRO_E_ARG, "hydro_check_status: no status buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, gr->status_dev, sizeof(flag), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (flag & HYDRO_STATUS_TABLE) return fail(HYDRO_E_TABLE, "neighbour table is inconsistent");
  if (flag & HYDRO_STATUS_UNPHYSICAL)
    return fail(HYDRO_E_UNPHYSICAL, "rho <= 0 or p <= 0 met at a face");
  return HYDRO_OK;
}

}  // extern "C"
