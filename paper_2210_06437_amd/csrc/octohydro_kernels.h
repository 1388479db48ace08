// Device code of liboctohydro shared by its translation units: constants,
// argument structs, the method's device functions, and the kernel templates
// with their launchers.  Each kernel is instantiated only in the translation
// unit that launches it (octohydro.hip: ghost fill, restriction, CFL, totals,
// flux correction; k_step_f64.hip, k_step_f32.hip and their _cfl and
// _restrict variants: the fused substep per precision and variant), so the
// units compile in parallel.  The 3D step's device code is in
// octohydro_kernels3d.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "octohydro.h"

namespace octohydro {

constexpr int SUB = 8;
constexpr int GH = 3;
constexpr int TW = SUB + 2 * GH;  // 14
constexpr int CELLS = SUB * SUB * SUB;
constexpr int TILE = TW * TW * TW;
constexpr int NF_CORE = 6;  // rho, sx, sy, sz, E, tau
constexpr int ACC_PITCH = 9;  // LDS row pitch (doubles) of the accumulator
constexpr int ACC_PLANE = SUB * ACC_PITCH;
// Bound on the byte size of every array the kernels address with 32-bit
// offsets (buffer resources and 32-bit lane offsets); checked on the host.
constexpr uint32_t OFF_NONE = 0xFFFFF000u;

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
  // flux register (NULL: no coarse-fine flux correction)
  const int32_t* face_slot;
  const int32_t* fine_slot;
  const int32_t* slot_leaf;
  double* reg;
  double omega;  // rotating-frame angular velocity (0: no sources)
  void* rstate;  // restricted copies of the refined nodes [nf][n_nodes][512]
  // node * 8 + octant of each leaf that is a child of a refined node, or -1
  const int32_t* leaf_node;
};

// Values per register slot and field: 64 coarse face fluxes, then the 16x16
// fine face fluxes that cover the same face.
constexpr int REG_COARSE = 64;
constexpr int REG_STRIDE = 64 + 256;

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

// ---------------------------------------------------------------------------
// Restricted copies of the refined nodes (the coarse side of a coarse-fine
// face, Sec. VI): coarse cell (x, y, z) of node n is the mean of the 8 cells
// of child (x>>2, y>>2, z>>2) that cover it, summed in the same fixed order as
// the ghost fill.  Cells of a missing child are never read; they are set to 0.
// ---------------------------------------------------------------------------
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  typedef double2 type;
};
template <>
struct Pair<float> {
  typedef float2 type;
};

// Workgroup (node, field) of 512 threads, thread = coarse cell; the two x
// neighbours of each fine pair are read as one aligned 2-element load.
template <typename T>
__global__ void __launch_bounds__(512)
    k_restrict(GridArgs g, const T* __restrict__ U, T* __restrict__ R) {
  typedef typename Pair<T>::type P;
  const int node = blockIdx.x, f = blockIdx.y, c = threadIdx.x;
  const int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
  const int child = g.children[8 * node + (z >> 2) * 4 + (y >> 2) * 2 + (x >> 2)];
  T v = T(0);
  if (child >= 0) {
    const T* u = U + (size_t)f * g.n_leaves * CELLS + (size_t)child * CELLS +
                 ((2 * z) & 7) * 64 + ((2 * y) & 7) * 8 + ((2 * x) & 7);
    const P a = *reinterpret_cast<const P*>(u), b = *reinterpret_cast<const P*>(u + 8),
            d = *reinterpret_cast<const P*>(u + 64), e = *reinterpret_cast<const P*>(u + 72);
    v = T(0.125) * (((a.x + a.y) + (b.x + b.y)) + ((d.x + d.y) + (e.x + e.y)));
  }
  R[((size_t)f * g.n_nodes + node) * CELLS + c] = v;
}

// ---------------------------------------------------------------------------
// PPM (Colella & Woodward 1984) as a streaming recurrence along a pencil.
// ---------------------------------------------------------------------------

// Keeps a value's computation ahead of this point in program order: an
// empty statement on a register (no instruction, no memory access).  The
// instruction selector otherwise orders pure arithmetic its own way and
// computes values long before their use, which holds registers: in the
// fused substep's stream step, binary64 at 11 fields took 420 registers
// with 179 AGPR moves per z-stream step and 356 with 68 with the pins.
// For 8-byte values the statement is volatile, which also keeps memory
// accesses from moving across it; for 4-byte values it is not, which lets
// the next group's loads start earlier: the binary32 3D step took 27.5 ms
// instead of 30.2, while the binary64 one was 1 % faster with the volatile
// form and the substep kernel the same either way (the same bits in all).
template <typename T>
__device__ __forceinline__ void keep_order(T& v) {
  if constexpr (sizeof(T) == 4)
    asm("" : "+v"(v));
  else
    asm volatile("" : "+v"(v));
}

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
  // min(2|dl|, 2|dr|) evaluated as 2 min(|dl|, |dr|): scaling by 2 is exact
  // and monotone, so both give the same bits
  const T lim = fmin(fabs(dq), T(2) * fmin(fabs(dl), fabs(dr)));
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
  // fix_l and fix_r exclude each other (dlr^2 >= 0, and a NaN makes both
  // false), so the right value needs no test of fix_l
  const T nl = flat ? c : (fix_l ? lo : l);
  const T nr = flat ? c : (fix_r ? ro : r);
  l = nl;
  r = nr;
}

// Feed the k-th value of a pencil stream; when k >= 5, returns the face
// states of the face between stream cells k-3 and k-2 in (UL, UR).  k is a
// compile-time constant after unrolling.
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

// Internal energy density from the entropy tracer, tau^gamma (dual-energy
// switch).  Kept out of line: the branch is rare and the inlined pow would
// hold registers in the hot loop.
static __device__ __noinline__ double tau_energy(double tau, double gamma) { return pow(tau, gamma); }
static __device__ __noinline__ float tau_energy(float tau, float gamma) { return powf(tau, gamma); }

// rinv = 1/rho, p, c for conserved state (rho, sx, sy, sz, E, tau).
template <typename T>
__device__ __forceinline__ bool eos(const Phys<T>& ph, T rho, T sx, T sy, T sz, T E, T tau,
                                    T& rinv, T& p, T& c) {
  rinv = T(1) / rho;
  const T ss = (sx * sx + sy * sy) + sz * sz;
  T ei = E - T(0.5) * ss * rinv;
  if (ei < ph.eta1 * E) ei = tau_energy(tau, ph.gamma);
  p = ph.gm1 * ei;
  c = sqrt(ph.gamma * p * rinv);
  return !(rho > T(0)) || !(p > T(0));
}

// ---------------------------------------------------------------------------
// Fused substep kernel
// ---------------------------------------------------------------------------

// Leaf of workgroup `bid` under the XCD remap mode (the hardware deals
// consecutive workgroups to the 8 XCDs in turn, so workgroup b runs on XCD
// b % 8 as its (b / 8)-th): 0 keeps b; 1 gives each XCD one contiguous
// range of leaves; c >= 2 deals chunks of c consecutive leaves to the XCDs
// in turn (leaves past the last whole round of 8 chunks keep b).  Leaves
// are stored in Morton order, so either keeps the leaves an XCD works on at
// once close in space and their halos in that XCD's L2.
__device__ __forceinline__ int leaf_of_block(int bid, int n, int remap) {
  if (remap == 1) {
    const int q = n >> 3, r = n & 7;
    const int xcd = bid & 7, j = bid >> 3;
    return xcd * q + min(xcd, r) + j;
  }
  if (remap >= 2) {
    const int round = 8 * remap;
    if (bid >= (n / round) * round) return bid;
    const int xcd = bid & 7, j = bid >> 3;
    return ((j / remap) * 8 + xcd) * remap + j % remap;
  }
  return bid;
}

struct StepArgs {
  GridArgs g;
  const void* U0;
  const void* Uk;
  void* Uout;
  const double* dt;
  double beta;
  int32_t leaf_base;  // first leaf (per-leaf launches); 0 for the batch
  int32_t remap;      // XCD remap mode of leaf_of_block
  // CFL epilogue: when set, the kernel also takes the minimum over its cells
  // of dx / (max|v| + c) of the values it stores (Sec. V-B-1: the substep
  // takes part in the global time-step size) into *dt_next (a binary64
  // whose bit pattern is reduced with an unsigned 64-bit atomic min)
  double* dt_next;
  // Restricted copies of the output: when set, every leaf that is a child of
  // a refined node also writes the coarse (8-cell mean) cells its output
  // covers into this [nf][n_nodes][512] array, in the order of the ghost
  // fill's restriction, for the next substep's refined-side ghosts.
  void* node_out;
};

// Kernel variants of the fused substep (see k_step).
constexpr int STEP_PLAIN = 0;
constexpr int STEP_RESTRICT = 1;
constexpr int STEP_CFL = 2;

// Coarse cell of node copy that leaf cell (x, y, z) lies in, for a leaf in
// octant `oct` (x + 2 y + 4 z of the child position) of its node.
__device__ __forceinline__ int coarse_cell(int oct, int x, int y, int z) {
  return (4 * (oct >> 2) + (z >> 1)) * 64 + (4 * ((oct >> 1) & 1) + (y >> 1)) * 8 +
         (4 * (oct & 1) + (x >> 1));
}

// Restriction of stored output values as a by-product of the Z phase.  Lane
// (x, y) finishes cells (x, y, z) for consecutive z; the 2x2 transverse sum
// of a plane, ((v(x) + v(x^1)) + (v(y^1) + v(x^1, y^1))), is the same in all
// four lanes of the group (both additions commute).  At even z it is parked
// in the cell's accumulator slot (read already); at odd z the parked sum of
// z - 1 and this plane's sum give the coarse value
// 0.125 * ((sum at z - 1) + (sum at z)), which the lane at even (x, y)
// stores.  That is 0.125 * (((v000 + v100) + (v010 + v110)) + ((v001 + v101)
// + (v011 + v111))), the ghost fill's order, in the element type.
// Value of lane ^ 1 (DPP quad permutation [1,0,3,2]) and of lane ^ 8 (DPP
// rotation by 8 within a row of 16 lanes): register moves between lanes,
// no LDS traffic.
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR8 = 0x128;

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <typename T, int PLANE>
__device__ __forceinline__ void restrict_out(const StepArgs& s, double* __restrict__ slot,
                                             int node, int f, int x, int y, int z, T o) {
  const T t = o + dpp_move<DPP_XOR1>(o);
  const T q = t + dpp_move<DPP_XOR8>(t);
  if ((z & 1) == 0) {
    *slot = (double)q;
  } else {
    const T r = T(0.125) * ((T)slot[-PLANE] + q);
    if (((x | y) & 1) == 0)
      static_cast<T*>(s.node_out)[((size_t)f * s.g.n_nodes + (node >> 3)) * CELLS +
                                  coarse_cell(node & 7, x, y, z)] = r;
  }
}

// Per-cell CFL quantity dx / (max(|v_x|, |v_y|, |v_z|) + c) of a stored
// state (rho, s, E, tau as stored, in binary64), evaluated operation by
// operation as the time-step pass hydro_cfl_dt does.
template <typename T>
__device__ __forceinline__ double cfl_quantity(const GridArgs& g, const T (&cv)[NF_CORE],
                                               double dx) {
  const double rho = (double)cv[0], sx = (double)cv[1], sy = (double)cv[2];
  const double sz = (double)cv[3], E = (double)cv[4];
  const double rinv = 1.0 / rho;
  const double ss = (sx * sx + sy * sy) + sz * sz;
  double ei = E - 0.5 * ss * rinv;
  if (ei < g.eta1 * E) ei = tau_energy((double)cv[5], g.gamma);
  const double p = (g.gamma - 1.0) * ei;
  const double c = sqrt(g.gamma * p * rinv);
  const double vmax = fmax(fmax(fabs(sx * rinv), fabs(sy * rinv)), fabs(sz * rinv));
  return dx / (vmax + c);
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Wavefront minimum of a positive binary64 into *out by an unsigned 64-bit
// atomic min on its bit pattern (positive doubles order like their bits).
__device__ __forceinline__ void atomic_min_positive(double* out, double v, int lane) {
  v = wave_min(v);
  if (lane == 0)
    atomicMin(reinterpret_cast<unsigned long long*>(out),
              (unsigned long long)__double_as_longlong(v));
}

// Per-leaf constants.  Neighbour kinds and ids of the six face neighbours are
// handed to the phases as plain values (the phase picks its axis once), so
// no per-lane choice is ever made by indexing memory.
struct LeafInfo {
  int leaf, blocks;
  int ix, iy, iz;
};

// Face neighbour (kind, id) of a pencil axis, low and high side.
struct FaceNbr {
  int klo, ilo, khi, ihi;
  int rlo, rhi;  // coarse register slot of the low / high face, or -1
  int flo, fhi;  // fine register entry (slot << 2 | quadrant), or -1
};

// Record the fluxes H (all fields) through face `face` (0 = low, 8 = high
// face of the leaf) of a pencil at transverse position (u, v) of that face.
template <typename T, int NF>
__device__ __forceinline__ void record_face(const GridArgs& g, const FaceNbr& fn, int face, int u,
                                            int v, const T (&H)[NF]) {
  const int cs = face == 0 ? fn.rlo : fn.rhi;
  const int fe = face == 0 ? fn.flo : fn.fhi;
  if (cs >= 0) {
    double* r = g.reg + (size_t)cs * NF * REG_STRIDE + u + 8 * v;
#pragma unroll
    for (int f = 0; f < NF; ++f) r[f * REG_STRIDE] = (double)H[f];
  }
  if (fe >= 0) {
    const int q = fe & 3;
    double* r = g.reg + (size_t)(fe >> 2) * NF * REG_STRIDE + REG_COARSE +
                (8 * (q & 1) + u) + 16 * (8 * (q >> 1) + v);
#pragma unroll
    for (int f = 0; f < NF; ++f) r[f * REG_STRIDE] = (double)H[f];
  }
}

// A lane's pencil along axis d through transverse cell (a, b): where each of
// its 14 stream values comes from, as byte offsets into a field array.
// Interior value k sits at off + (k-3) sd; each ghost value k in
// {0,1,2,11,12,13} comes from gofs[] -- a same-level cell or the covering
// coarse cell (injection) of the state, or, on a refined side (ref_lo /
// ref_hi), a cell of the refined node's restricted copy.  The sources are the
// same for every field, so they are worked out once per pencil.
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

struct Pencil {
  uint32_t off, sd;
  u32x8 gofs;  // a vector value: selecting an entry never touches memory
  bool ref_lo, ref_hi;
  bool any_lo, any_hi;  // some lane of the wave has ref_lo (ref_hi)
};

// cd = the leaf's block coordinate along d.
__device__ __forceinline__ uint32_t ghost_offset(const GridArgs& g, const LeafInfo& li, int kind,
                                                 int id, int side, int d, int cd, int lx, int ly,
                                                 int lz) {
  if (kind == HYDRO_SAME_LEAF) return id * CELLS + lz * 64 + ly * 8 + lx;
  if (kind == HYDRO_COARSER_LEAF) {
    // the neighbour block along d, wrapped; transverse blocks are the leaf's
    const int nb = wrap(cd + side, li.blocks);
    const int bx = d == 0 ? nb : li.ix, by = d == 1 ? nb : li.iy, bz = d == 2 ? nb : li.iz;
    return id * CELLS + (4 * (bz & 1) + (lz >> 1)) * 64 + (4 * (by & 1) + (ly >> 1)) * 8 +
           (4 * (bx & 1) + (lx >> 1));
  }
  // refined neighbour: the coarse cell of the node's restricted copy
  return id * CELLS + lz * 64 + ly * 8 + lx;
}

template <typename T>
__device__ __forceinline__ Pencil make_pencil(const GridArgs& g, const LeafInfo& li, int d, int a,
                                              int b, const FaceNbr& fn) {
  Pencil p;
  constexpr uint32_t W = sizeof(T);
  // d = 0: (x, a=y, b=z); d = 1: (a=x, y, b=z); d = 2: (a=x, b=y, z)
  p.off = W * (li.leaf * CELLS + (d == 0 ? b * 64 + a * 8 : (d == 1 ? b * 64 + a : b * 8 + a)));
  p.sd = W * (d == 0 ? 1 : (d == 1 ? 8 : 64));
  const int klo = fn.klo, ilo = fn.ilo, khi = fn.khi, ihi = fn.ihi;
  p.ref_lo = klo == HYDRO_SAME_REFINED;
  p.ref_hi = khi == HYDRO_SAME_REFINED;
  // wave votes taken once per pencil, outside the streaming loops
  p.any_lo = __any(p.ref_lo);
  p.any_hi = __any(p.ref_hi);
  // the block coordinate along d (d may differ between lanes), as arithmetic
  // on values: a select between the LeafInfo fields became an indexed load
  // from a scratch copy of it, with a full memory wait per ghost position
  const int cd = (d == 0) * li.ix + (d == 1) * li.iy + (d == 2) * li.iz;
#pragma unroll
  for (int j = 0; j < 2 * GH; ++j) {
    const bool hi = j >= GH;
    const int l = hi ? j - GH : j + SUB - GH;  // cell along d inside the neighbour block
    const int lx = d == 0 ? l : a;
    const int ly = d == 0 ? a : (d == 1 ? l : b);
    const int lz = d == 2 ? l : b;
    p.gofs[j] =
        W * ghost_offset(g, li, hi ? khi : klo, hi ? ihi : ilo, hi ? 1 : -1, d, cd, lx, ly, lz);
  }
  return p;
}

// Where stream position k (0..13) of a pencil comes from: a byte offset
// into a field array and whether it is a refined ghost (mean of 8 cells).
// Worked out once per stream step and shared by every field; for a step
// index known only at run time the ghost offset is picked by a select chain
// over the six values.
struct Src {
  uint32_t o;    // offset of the value in its array
  bool ref;      // this lane's value comes from a node copy
  bool any_ref;  // some lane of the wave reads a node copy (wave-uniform)
};

__device__ __forceinline__ Src pencil_src(const Pencil& p, int k) {
  Src s;
  if (k >= GH && k < GH + SUB) {
    s.o = p.off + (uint32_t)(k - GH) * p.sd;
    s.ref = s.any_ref = false;
    return s;
  }
  s.o = k == 0 ? p.gofs[0] : k == 1 ? p.gofs[1] : k == 2 ? p.gofs[2]
      : k == 11 ? p.gofs[3] : k == 12 ? p.gofs[4] : p.gofs[5];
  s.ref = k < GH ? p.ref_lo : p.ref_hi;
  s.any_ref = k < GH ? p.any_lo : p.any_hi;
  return s;
}

// Buffer view of a state array: a 128-bit resource (base address, size)
// held in scalar registers.  A load names the field by a scalar byte offset
// (f times the field stride) and the cell by a 32-bit lane byte offset plus
// a small immediate, so no 64-bit per-lane address is ever formed.  The
// whole array must stay below 4 GiB (checked on the host).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int RSRC_WORD3 = 0x00020000;  // raw dword data format (gfx9 family)

__device__ __forceinline__ Rsrc state_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, RSRC_WORD3);
}

// Field view: the array's resource and the field's scalar byte offset.
struct FieldView {
  Rsrc r;
  uint32_t fo;
};

__device__ __forceinline__ double bload(double, const FieldView& v, uint32_t o) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v.r, (int)o, (int)v.fo, 0));
}
__device__ __forceinline__ float bload(float, const FieldView& v, uint32_t o) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v.r, (int)o, (int)v.fo, 0));
}
// A value read once and by no other leaf (U0): loaded with the non-temporal
// cache policy (bit 1 of the buffer instruction's cache-policy operand on
// gfx950), so that it does not push halo values out of the L2 (measured
// about -1 % on the FP64 substep of the 65535-leaf case).
constexpr int CACHE_NT = 2;
__device__ __forceinline__ double bload_once(double, const FieldView& v, uint32_t o) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(v.r, (int)o, (int)v.fo, CACHE_NT));
}
__device__ __forceinline__ float bload_once(float, const FieldView& v, uint32_t o) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_raw_buffer_load_b32(v.r, (int)o, (int)v.fo, CACHE_NT));
}

// The two arrays stream values come from: the stage input (all interior and
// same-level or coarser ghosts) and the restricted node copies (ghosts on a
// refined side), each with its field stride in bytes.
struct Sources {
  Rsrc uk, rn;
  uint32_t uk_fs, rn_fs;
};

__device__ __forceinline__ Sources make_sources(const void* Uk, const void* rstate, int nf,
                                                uint32_t uk_fs, uint32_t rn_fs) {
  return Sources{state_rsrc(Uk, (uint32_t)nf * uk_fs),
                 state_rsrc(rstate, rstate ? (uint32_t)nf * rn_fs : 0u), uk_fs, rn_fs};
}

// The values of a stream position in all NF fields.  Where some lane of the
// wave reads a node copy, the lanes read from two arrays: the lanes of each
// array load under their own execution mask into the same registers, all
// fields issued before any is used, with no select.  (Two loads per field,
// one of them past the end of its array, and a select took two registers
// per field and made the compiler serialise the loads with a full memory
// wait per field: 11 memory latencies per such position.)  The test is
// made once per position, not once per field.
template <typename T, int NF>
__device__ __forceinline__ void load_position(const Sources& S, const Src& s, T (&q)[NF]) {
  if (s.any_ref) {
    if (s.ref) {
#pragma unroll
      for (int f = 0; f < NF; ++f) q[f] = bload(T(), FieldView{S.rn, f * S.rn_fs}, s.o);
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) q[f] = bload(T(), FieldView{S.uk, f * S.uk_fs}, s.o);
    }
  } else {
#pragma unroll
    for (int f = 0; f < NF; ++f) q[f] = bload(T(), FieldView{S.uk, f * S.uk_fs}, s.o);
  }
}

// Kurganov-Tadmor fluxes of the core fields at one face normal to axis d;
// also returns the face's normal velocities and half the signal speed for
// the passive species.
template <typename T>
__device__ __forceinline__ void core_flux(const Phys<T>& ph, int d, const T (&UL)[NF_CORE],
                                          const T (&UR)[NF_CORE], T (&H)[NF_CORE], T& vL, T& vR,
                                          T& ha, bool& bad) {
  T riL, pL, cL, riR, pR, cR;
  bad |= eos(ph, UL[0], UL[1], UL[2], UL[3], UL[4], UL[5], riL, pL, cL);
  bad |= eos(ph, UR[0], UR[1], UR[2], UR[3], UR[4], UR[5], riR, pR, cR);
  const T snL = d == 0 ? UL[1] : (d == 1 ? UL[2] : UL[3]);
  const T snR = d == 0 ? UR[1] : (d == 1 ? UR[2] : UR[3]);
  vL = snL * riL;
  vR = snR * riR;
  ha = T(0.5) * fmax(fabs(vL) + cL, fabs(vR) + cR);
  T FL[NF_CORE], FR[NF_CORE];
  FL[0] = snL;
  FR[0] = snR;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const T fl = UL[1 + m] * vL;
    const T fr = UR[1 + m] * vR;
    FL[1 + m] = m == d ? fl + pL : fl;
    FR[1 + m] = m == d ? fr + pR : fr;
  }
  FL[4] = (UL[4] + pL) * vL;
  FR[4] = (UR[4] + pR) * vR;
  FL[5] = UL[5] * vL;
  FR[5] = UR[5] * vR;
#pragma unroll
  for (int f = 0; f < NF_CORE; ++f) H[f] = T(0.5) * (FL[f] + FR[f]) - ha * (UR[f] - UL[f]);
}

// Stage combination of one cell: t = Uk + dt L with L = -sum * inv_dx, then
// t (first stage) or U0 + beta (t - U0); u0 is the cell's U0 value, loaded
// by the caller ahead of time.
template <typename T>
__device__ __forceinline__ T finish_cell(const StepArgs& s, size_t fbase, uint32_t cell, T uk,
                                         T u0, double sum, bool has_src, double src, double dt,
                                         double inv_dx) {
  double lrate = -sum * inv_dx;
  if (has_src) lrate = lrate + src;
  const double t = (double)uk + dt * lrate;
  double out;
  if (s.U0) {
    const double u = (double)u0;
    out = u + s.beta * (t - u);
  } else {
    out = t;
  }
  // the result is not read again by this kernel: keep it out of the caches
  __builtin_nontemporal_store((T)out, static_cast<T*>(s.Uout) + fbase + cell);
  return (T)out;
}

// Scheduling fence between the per-field reconstructions of a stream step:
// the fields are then evaluated one after another instead of interleaved,
// which keeps fewer temporaries alive (measured: FP32 -7 %, FP64 neutral).
#ifndef OCTOHYDRO_FENCE_FIELDS
#define OCTOHYDRO_FENCE_FIELDS 1
#endif
#if OCTOHYDRO_FENCE_FIELDS
#define OCTOHYDRO_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define OCTOHYDRO_FENCE() ((void)0)
#endif

// LDS accumulator of half a leaf (4 z-planes): field stride ACC_HALF.
constexpr int ACC_HALF = 4 * ACC_PLANE;

// The same layout with row pitch AP (doubles).  AP = 9, the spare double per
// row, puts the 8 lanes of an x-pencil group, which add into the same x of 8
// rows, on distinct LDS banks; AP = 8 takes 11 % less LDS.  With the 256-
// register budget the accumulator is what limits the workgroups per CU
// (binary64 at 11 fields: 25.3 KB, 6 per CU; 22.5 KB with AP = 8, 7 per CU):
// there AP = 8 made the binary32 substep of the 65,535-leaf case 8.5 % faster
// (3.19 -> 2.92 ms); with the 512-register budget, where registers limit it
// to 4 per CU, AP = 9 is 0.8 % faster.  The accumulator sums two exact
// terms, so the layout does not change a bit of the result.
template <int AP>
struct AccLayout {
  static constexpr int PITCH = AP, PLANE = SUB * AP, HALF = 4 * SUB * AP;
};

// Point after which lanes of a wave read LDS values that other lanes of the
// same wave wrote.  One wave's LDS instructions execute in program order, so
// the hardware needs no wait; the wavefront-scope fences (which emit no
// instructions) keep the compiler from moving memory accesses across the
// point, which the wave barrier alone does not.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First five stream steps of all NF fields of a pencil (stream positions
// k0..k0+4): they build the PPM recurrences up to the first complete cell;
// no face is complete yet.  Unrolled, so each step does only the work its
// stencil allows.
template <typename T, int NF>
__device__ __forceinline__ void stream_prologue(Ppm<T> (&st)[NF], const Sources& S,
                                                const Pencil& p, int k0) {
  // one position in flight ahead of the recurrences
  T cur[NF], nxt[NF];
  load_position<T, NF>(S, pencil_src(p, k0), cur);
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    if (j + 1 < 5) load_position<T, NF>(S, pencil_src(p, k0 + j + 1), nxt);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      T ul, ur;
      ppm_push(st[f], cur[f], j, ul, ur);
      cur[f] = nxt[f];
    }
  }
}

// A steady stream step: feed the next value of every field and evaluate the
// face between stream cells k-3 and k-2 (fluxes in H).  The core fields are
// reconstructed first and give the face's velocities and signal speed; each
// passive species is then reconstructed and fluxed on its own, so only one
// species' face states are ever held at a time.
template <typename T, int NF>
__device__ __forceinline__ void stream_step(const Phys<T>& ph, int d, Ppm<T> (&st)[NF],
                                            const T (&qn)[NF], T (&H)[NF], bool& bad) {
  T core_L[NF_CORE], core_R[NF_CORE], Hc[NF_CORE], vL, vR, ha;
#pragma unroll
  for (int f = 0; f < NF_CORE; ++f) {
    ppm_push(st[f], qn[f], 5, core_L[f], core_R[f]);
    keep_order(core_L[f]);
    keep_order(core_R[f]);
    keep_order(st[f].Rprev);
    keep_order(st[f].qfA);
    keep_order(st[f].dmA);
    OCTOHYDRO_FENCE();
  }
  core_flux(ph, d, core_L, core_R, Hc, vL, vR, ha, bad);
  keep_order(vL);
  keep_order(vR);
  keep_order(ha);
#pragma unroll
  for (int f = 0; f < NF_CORE; ++f) {
    H[f] = Hc[f];
    keep_order(H[f]);
  }
#pragma unroll
  for (int f = NF_CORE; f < NF; ++f) {
    OCTOHYDRO_FENCE();
    T ul, ur;
    ppm_push(st[f], qn[f], 5, ul, ur);
    H[f] = T(0.5) * (ul * vL + ur * vR) - ha * (ur - ul);
    keep_order(H[f]);
    keep_order(st[f].Rprev);
    keep_order(st[f].qfA);
    keep_order(st[f].dmA);
  }
}

// Phase XY of half h: lanes 0-31 stream x-pencils, lanes 32-63 y-pencils of
// the planes z in [4h, 4h+4).  Each cell receives dHx from one lane and dHy
// from another, both as LDS atomic adds (ds_add_f64, which rounds as binary64
// addition does) into an accumulator cleared to -0.0: -0.0 is the identity of
// binary64 addition (it keeps the sign of a zero term) and a sum of two terms
// does not depend on their order, so the accumulator holds exactly dHx + dHy
// whichever lane gets there first, with no branch on the lane.
template <typename T, int NF, int AP>
__device__ __forceinline__ void phase_xy(const StepArgs& s, const Phys<T>& ph, const LeafInfo& li,
                                         const FaceNbr& fn, double* __restrict__ acc, int h,
                                         int lane, bool& bad) {
  const GridArgs& g = s.g;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const uint32_t fs_b = (uint32_t)(fs * sizeof(T));
  const uint32_t rn_fs = (uint32_t)((size_t)g.n_nodes * CELLS * sizeof(T));
  const Sources S = make_sources(s.Uk, g.rstate, g.nf, fs_b, rn_fs);
  const int d = lane >> 5;
  const int a = lane & 7;
  const int zz = (lane >> 3) & 3;
  const Pencil p = make_pencil<T>(g, li, d, a, 4 * h + zz, fn);
  using L = AccLayout<AP>;
  const int acc_off = d == 0 ? zz * L::PLANE + a * L::PITCH : zz * L::PLANE + a;
  const int acc_step = d == 0 ? 1 : L::PITCH;

  for (int j = lane; j < NF * L::HALF / 2; j += 64)
    reinterpret_cast<double2*>(acc)[j] = make_double2(-0.0, -0.0);
  wave_lds_sync();
  Ppm<T> st[NF];
  double Hprev[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    st[f] = Ppm<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    Hprev[f] = 0.0;
  }
  stream_prologue<T, NF>(st, S, p, 0);
  T qnext[NF];
  load_position<T, NF>(S, pencil_src(p, 5), qnext);
#pragma unroll 1
  for (int k = 5; k < TW; ++k) {
    T qn[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) qn[f] = qnext[f];
    if (k + 1 < TW) load_position<T, NF>(S, pencil_src(p, k + 1), qnext);
    T H[NF];
    stream_step<T, NF>(ph, d, st, qn, H, bad);
    if (g.reg && (k == 5 || k == TW - 1)) record_face<T, NF>(g, fn, k - 5, a, 4 * h + zz, H);
    if (k >= 6) {
      const int i = k - 6;  // interior cell along d: H now is its high face
      const int ai = acc_off + i * acc_step;
      double dH[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) dH[f] = (double)H[f] - Hprev[f];
#pragma unroll
      for (int f = 0; f < NF; ++f)
        __hip_atomic_fetch_add(&acc[f * L::HALF + ai], dH[f], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) Hprev[f] = (double)H[f];
  }
}

// Phase Z of half h: lane (x, y) streams its z-pencil over stream positions
// [4h, 4h+10), which yields the z-faces of cells z in [4h, 4h+4), adds dHz
// to the accumulator and finishes those cells.  ZU: unroll factor of the
// stream loop.  Unrolled by 2, consecutive steps keep the stream state in
// alternating registers instead of copying it back at every step: with the
// 512-register budget that was 2-3 % faster in binary64 (the same bits); at
// two wavefronts per SIMD it was 1 % slower.
template <typename T, int NF, int MODE, int ZU, int AP>
__device__ __forceinline__ void phase_z(const StepArgs& s, const Phys<T>& ph, const LeafInfo& li,
                                        const FaceNbr& fn, double* __restrict__ acc, int h,
                                        int lane, double dt, double inv_dx, bool& bad,
                                        double& cflmin, int lnode) {
  const GridArgs& g = s.g;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const uint32_t fs_b = (uint32_t)(fs * sizeof(T));
  const uint32_t rn_fs = (uint32_t)((size_t)g.n_nodes * CELLS * sizeof(T));
  const Sources S = make_sources(s.Uk, g.rstate, g.nf, fs_b, rn_fs);
  const Rsrc U0 = state_rsrc(s.U0 ? s.U0 : s.Uk, (uint32_t)(g.nf * fs * sizeof(T)));
  const int x = lane & 7, y = lane >> 3;
  const Pencil p = make_pencil<T>(g, li, 2, x, y, fn);
  const int k0 = 4 * h;
  const uint32_t leaf_at = (uint32_t)li.leaf * CELLS + y * 8 + x;

  Ppm<T> st[NF];
  double Hprev[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    st[f] = Ppm<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    Hprev[f] = 0.0;
  }
  stream_prologue<T, NF>(st, S, p, k0);
  T qnext[NF];
  load_position<T, NF>(S, pencil_src(p, k0 + 5), qnext);
#pragma unroll ZU
  for (int kk = 5; kk < 10; ++kk) {
    const int k = k0 + kk;
    T qn[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) qn[f] = qnext[f];
    if (kk + 1 < 10) load_position<T, NF>(S, pencil_src(p, k + 1), qnext);
    // U0 of the cell this step finishes: issued now, consumed after the
    // face evaluation, so the load's latency is covered by it
    T u0v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) u0v[f] = T(0);
    if (kk >= 6 && s.U0) {
      const uint32_t cell_b = (uint32_t)sizeof(T) * (leaf_at + (k - 6) * 64);
#pragma unroll
      for (int f = 0; f < NF; ++f) u0v[f] = bload_once(T(), FieldView{U0, f * fs_b}, cell_b);
    }
    T H[NF];
    stream_step<T, NF>(ph, 2, st, qn, H, bad);
    if (g.reg && (k == 5 || k == TW - 1)) record_face<T, NF>(g, fn, k - 5, x, y, H);
    if (kk >= 6) {
      const int i = k - 6;  // interior cell along z
      using L = AccLayout<AP>;
      const int ai = (i - k0) * L::PLANE + y * L::PITCH + x;
      // rotating-frame sources of s_x, s_y, s_z, E from this cell's Uk
      double src[4] = {0.0, 0.0, 0.0, 0.0};
      const bool rot = g.omega != 0.0;
      if (rot) {
        const double dx = 1.0 / (double)(SUB * li.blocks);
        const double rx = ((double)(SUB * li.ix + x) + 0.5) * dx - 0.5;
        const double ry = ((double)(SUB * li.iy + y) + 0.5) * dx - 0.5;
        const double rho = (double)st[0].qy, sx = (double)st[1].qy, sy = (double)st[2].qy;
        const double om2 = g.omega * g.omega, tw = 2.0 * g.omega;
        src[0] = tw * sy + rho * om2 * rx;
        src[1] = rho * om2 * ry - tw * sx;
        src[3] = om2 * (sx * rx + sy * ry);
      }
      T cv[NF_CORE];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double sum = acc[f * L::HALF + ai] + ((double)H[f] - Hprev[f]);
        const T o = finish_cell<T>(s, (size_t)f * fs, leaf_at + i * 64, st[f].qy, u0v[f], sum,
                                   rot && f >= 1 && f <= 4, f >= 1 && f <= 4 ? src[f - 1] : 0.0,
                                   dt, inv_dx);
        if (f < NF_CORE) cv[f] = o;
        if constexpr (MODE == STEP_RESTRICT) {
          if (lnode >= 0)
            restrict_out<T, L::PLANE>(s, &acc[f * L::HALF + ai], lnode, f, x, y, i, o);
        }
      }
      if constexpr (MODE == STEP_CFL) cflmin = fmin(cflmin, cfl_quantity<T>(g, cv, 1.0 / inv_dx));
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) Hprev[f] = (double)H[f];
  }
}

// W = register budget: W waves per SIMD (1: up to 512 VGPRs, 2: up to 256).
// MODE: STEP_PLAIN, STEP_RESTRICT (s.node_out set: the node copies of the
// output are left as well) or STEP_CFL (s.dt_next set: the CFL minimum of
// the output is taken as well); separate kernels, so that each keeps only
// the registers its own work needs.
template <typename T, int NF, int W, int MODE>
__global__ void __launch_bounds__(64, W) k_step(StepArgs s) {
  constexpr int AP = W == 2 ? 8 : 9;  // accumulator row pitch (see AccLayout)
  __shared__ __align__(16) double acc[NF * AccLayout<AP>::HALF];
  const GridArgs& g = s.g;
  const int leaf = s.leaf_base + leaf_of_block(blockIdx.x, g.n_leaves, s.remap);
  if (leaf >= g.n_leaves) return;
  const int lane = threadIdx.x;

  LeafInfo li;
  li.leaf = leaf;
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  li.ix = c4.y;
  li.iy = c4.z;
  li.iz = c4.w;
  li.blocks = g.base << c4.x;
  // face-neighbour slots: -x 12, +x 14, -y 10, +y 16, -z 4, +z 22
  const uint8_t* kd = g.kind + 27 * leaf;
  const int32_t* nb = g.nbr + 27 * leaf;
  const bool xlane = lane < 32;  // phase XY: lanes 0-31 x-pencils, 32-63 y-pencils
  FaceNbr fxy, fz;
  fxy.klo = xlane ? (int)kd[12] : (int)kd[10];
  fxy.ilo = xlane ? nb[12] : nb[10];
  fxy.khi = xlane ? (int)kd[14] : (int)kd[16];
  fxy.ihi = xlane ? nb[14] : nb[16];
  fz.klo = kd[4];
  fz.ilo = nb[4];
  fz.khi = kd[22];
  fz.ihi = nb[22];
  fxy.rlo = fxy.rhi = fxy.flo = fxy.fhi = -1;
  fz.rlo = fz.rhi = fz.flo = fz.fhi = -1;
  if (g.reg) {
    // register slots per face orientation o = 2*axis + side
    const int32_t* fsl = g.face_slot + 6 * leaf;
    const int32_t* fin = g.fine_slot + 6 * leaf;
    fxy.rlo = xlane ? fsl[0] : fsl[2];
    fxy.rhi = xlane ? fsl[1] : fsl[3];
    fxy.flo = xlane ? fin[0] : fin[2];
    fxy.fhi = xlane ? fin[1] : fin[3];
    fz.rlo = fsl[4];
    fz.rhi = fsl[5];
    fz.flo = fin[4];
    fz.fhi = fin[5];
  }
  const double dt = *s.dt;
  const double inv_dx = (double)(SUB * li.blocks);
  Phys<T> ph;
  ph.gamma = (T)g.gamma;
  ph.gm1 = (T)(g.gamma - 1.0);
  ph.eta1 = (T)g.eta1;

  bool bad = false;
  double cflmin = INFINITY;
  const int lnode = MODE == STEP_RESTRICT ? g.leaf_node[leaf] : -1;
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    phase_xy<T, NF, AP>(s, ph, li, fxy, acc, h, lane, bad);
    wave_lds_sync();
    phase_z<T, NF, MODE, W == 1 ? 2 : 1, AP>(s, ph, li, fz, acc, h, lane, dt, inv_dx, bad, cflmin,
                                             lnode);
    wave_lds_sync();
  }
  if constexpr (MODE == STEP_CFL) atomic_min_positive(s.dt_next, cflmin, lane);
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
}

// ---------------------------------------------------------------------------
// Two wavefronts per leaf.  The fields of a leaf are split between the two
// wavefronts of a 128-thread workgroup: wavefront 0 streams the six core
// fields (rho, s, E, tau) and evaluates the EOS and the Kurganov-Tadmor core
// flux at every face, wavefront 1 streams the passive species.  A species
// flux needs the face's normal velocities and half its signal speed, which
// wavefront 0 hands over through LDS: a double buffer whose slot alternates
// with every stream step of the leaf, one workgroup barrier per step (the
// slot wavefront 0 fills next was read by wavefront 1 before it reached the
// barrier that wavefront 0 has just passed).  Each wavefront accumulates and
// finishes its own fields (disjoint LDS accumulator ranges, wave-local
// hand-offs), so a field's arithmetic is exactly that of k_step.  Half the
// fields per wavefront halves the register set, which lets two wavefronts
// share a SIMD and hide each other's memory and dependency latency.
// ---------------------------------------------------------------------------

template <typename T>
struct SpeedSlot {
  T v[3][64];  // normal velocity left, right, half the signal speed; per lane
};

// Stream values of fields [F0, F0 + NG) at one position (see load_position).
template <typename T, int F0, int NG>
__device__ __forceinline__ void load_group(const Sources& S, const Src& s, T (&q)[NG]) {
  if (s.any_ref) {
    if (s.ref) {
#pragma unroll
      for (int i = 0; i < NG; ++i) q[i] = bload(T(), FieldView{S.rn, (F0 + i) * S.rn_fs}, s.o);
    } else {
#pragma unroll
      for (int i = 0; i < NG; ++i) q[i] = bload(T(), FieldView{S.uk, (F0 + i) * S.uk_fs}, s.o);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NG; ++i) q[i] = bload(T(), FieldView{S.uk, (F0 + i) * S.uk_fs}, s.o);
  }
}

template <typename T, int F0, int NG>
__device__ __forceinline__ void prologue_group(Ppm<T> (&st)[NG], const Sources& S,
                                               const Pencil& p, int k0) {
  T cur[NG], nxt[NG];
  load_group<T, F0, NG>(S, pencil_src(p, k0), cur);
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    if (j + 1 < 5) load_group<T, F0, NG>(S, pencil_src(p, k0 + j + 1), nxt);
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      T ul, ur;
      ppm_push(st[f], cur[f], j, ul, ur);
      cur[f] = nxt[f];
    }
  }
}

// Fluxes of fields [F0, F0 + NG) through face `face` of a pencil, recorded
// for the coarse-fine correction (see record_face).
template <typename T, int NF, int F0, int NG>
__device__ __forceinline__ void record_group(const GridArgs& g, const FaceNbr& fn, int face,
                                             int u, int v, const T (&H)[NG]) {
  const int cs = face == 0 ? fn.rlo : fn.rhi;
  const int fe = face == 0 ? fn.flo : fn.fhi;
  if (cs >= 0) {
    double* r = g.reg + (size_t)cs * NF * REG_STRIDE + u + 8 * v;
#pragma unroll
    for (int f = 0; f < NG; ++f) r[(F0 + f) * REG_STRIDE] = (double)H[f];
  }
  if (fe >= 0) {
    const int q = fe & 3;
    double* r = g.reg + (size_t)(fe >> 2) * NF * REG_STRIDE + REG_COARSE +
                (8 * (q & 1) + u) + 16 * (8 * (q >> 1) + v);
#pragma unroll
    for (int f = 0; f < NG; ++f) r[(F0 + f) * REG_STRIDE] = (double)H[f];
  }
}

// One steady stream step of a wavefront's field group: feed qn, evaluate the
// face (core group: EOS + core flux, speeds handed over; species group:
// speeds taken over) and return the group's fluxes in H.  Exactly one
// workgroup barrier per call in either group.
template <typename T, int F0, int NG>
__device__ __forceinline__ void group_step(const Phys<T>& ph, int d, Ppm<T> (&st)[NG],
                                           const T (&qn)[NG], T (&H)[NG],
                                           SpeedSlot<T>* __restrict__ spd, int slot, int lane,
                                           bool& bad) {
  if constexpr (F0 == 0) {
    static_assert(NG == NF_CORE, "the core group is the six core fields");
    T core_L[NF_CORE], core_R[NF_CORE], vL, vR, ha;
#pragma unroll
    for (int f = 0; f < NF_CORE; ++f) {
      ppm_push(st[f], qn[f], 5, core_L[f], core_R[f]);
      OCTOHYDRO_FENCE();
    }
    core_flux(ph, d, core_L, core_R, H, vL, vR, ha, bad);
    spd[slot].v[0][lane] = vL;
    spd[slot].v[1][lane] = vR;
    spd[slot].v[2][lane] = ha;
    __syncthreads();
  } else {
    T ul[NG], ur[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) {
      ppm_push(st[f], qn[f], 5, ul[f], ur[f]);
      OCTOHYDRO_FENCE();
    }
    __syncthreads();
    const T vL = spd[slot].v[0][lane], vR = spd[slot].v[1][lane], ha = spd[slot].v[2][lane];
#pragma unroll
    for (int f = 0; f < NG; ++f)
      H[f] = T(0.5) * (ul[f] * vL + ur[f] * vR) - ha * (ur[f] - ul[f]);
  }
}

// Phase XY of half h for one field group (see phase_xy).
template <typename T, int NF, int F0, int NG>
__device__ __forceinline__ void phase_xy_group(const StepArgs& s, const Phys<T>& ph,
                                               const LeafInfo& li, const FaceNbr& fn,
                                               double* __restrict__ acc,
                                               SpeedSlot<T>* __restrict__ spd, int& sn, int h,
                                               int lane, bool& bad) {
  const GridArgs& g = s.g;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const uint32_t fs_b = (uint32_t)(fs * sizeof(T));
  const uint32_t rn_fs = (uint32_t)((size_t)g.n_nodes * CELLS * sizeof(T));
  const Sources S = make_sources(s.Uk, g.rstate, g.nf, fs_b, rn_fs);
  const int d = lane >> 5;
  const int a = lane & 7;
  const int zz = (lane >> 3) & 3;
  const Pencil p = make_pencil<T>(g, li, d, a, 4 * h + zz, fn);
  const int acc_off = d == 0 ? zz * ACC_PLANE + a * ACC_PITCH : zz * ACC_PLANE + a;
  const int acc_step = d == 0 ? 1 : ACC_PITCH;

  double2* mine = reinterpret_cast<double2*>(acc + F0 * ACC_HALF);
  for (int j = lane; j < NG * ACC_HALF / 2; j += 64) mine[j] = make_double2(-0.0, -0.0);
  wave_lds_sync();
  Ppm<T> st[NG];
  double Hprev[NG];
#pragma unroll
  for (int f = 0; f < NG; ++f) {
    st[f] = Ppm<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    Hprev[f] = 0.0;
  }
  prologue_group<T, F0, NG>(st, S, p, 0);
  T qnext[NG];
  load_group<T, F0, NG>(S, pencil_src(p, 5), qnext);
#pragma unroll 1
  for (int k = 5; k < TW; ++k) {
    T qn[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) qn[f] = qnext[f];
    if (k + 1 < TW) load_group<T, F0, NG>(S, pencil_src(p, k + 1), qnext);
    T H[NG];
    group_step<T, F0, NG>(ph, d, st, qn, H, spd, sn & 1, lane, bad);
    ++sn;
    if (g.reg && (k == 5 || k == TW - 1))
      record_group<T, NF, F0, NG>(g, fn, k - 5, a, 4 * h + zz, H);
    if (k >= 6) {
      const int ai = acc_off + (k - 6) * acc_step;
      double dH[NG];
#pragma unroll
      for (int f = 0; f < NG; ++f) dH[f] = (double)H[f] - Hprev[f];
#pragma unroll
      for (int f = 0; f < NG; ++f)
        __hip_atomic_fetch_add(&acc[(F0 + f) * ACC_HALF + ai], dH[f], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
#pragma unroll
    for (int f = 0; f < NG; ++f) Hprev[f] = (double)H[f];
  }
}

// Phase Z of half h for one field group (see phase_z); the core group adds
// the rotating-frame sources.
template <typename T, int NF, int F0, int NG, int MODE>
__device__ __forceinline__ void phase_z_group(const StepArgs& s, const Phys<T>& ph,
                                              const LeafInfo& li, const FaceNbr& fn,
                                              double* __restrict__ acc,
                                              SpeedSlot<T>* __restrict__ spd, int& sn, int h,
                                              int lane, double dt, double inv_dx, bool& bad,
                                              double& cflmin, int lnode) {
  const GridArgs& g = s.g;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const uint32_t fs_b = (uint32_t)(fs * sizeof(T));
  const uint32_t rn_fs = (uint32_t)((size_t)g.n_nodes * CELLS * sizeof(T));
  const Sources S = make_sources(s.Uk, g.rstate, g.nf, fs_b, rn_fs);
  const Rsrc U0 = state_rsrc(s.U0 ? s.U0 : s.Uk, (uint32_t)(g.nf * fs * sizeof(T)));
  const int x = lane & 7, y = lane >> 3;
  const Pencil p = make_pencil<T>(g, li, 2, x, y, fn);
  const int k0 = 4 * h;
  const uint32_t leaf_at = (uint32_t)li.leaf * CELLS + y * 8 + x;

  Ppm<T> st[NG];
  double Hprev[NG];
#pragma unroll
  for (int f = 0; f < NG; ++f) {
    st[f] = Ppm<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    Hprev[f] = 0.0;
  }
  prologue_group<T, F0, NG>(st, S, p, k0);
  T qnext[NG];
  load_group<T, F0, NG>(S, pencil_src(p, k0 + 5), qnext);
#pragma unroll 1
  for (int kk = 5; kk < 10; ++kk) {
    const int k = k0 + kk;
    T qn[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) qn[f] = qnext[f];
    if (kk + 1 < 10) load_group<T, F0, NG>(S, pencil_src(p, k + 1), qnext);
    T u0v[NG];
#pragma unroll
    for (int f = 0; f < NG; ++f) u0v[f] = T(0);
    if (kk >= 6 && s.U0) {
      const uint32_t cell_b = (uint32_t)sizeof(T) * (leaf_at + (k - 6) * 64);
#pragma unroll
      for (int f = 0; f < NG; ++f)
        u0v[f] = bload_once(T(), FieldView{U0, (F0 + f) * fs_b}, cell_b);
    }
    T H[NG];
    group_step<T, F0, NG>(ph, 2, st, qn, H, spd, sn & 1, lane, bad);
    ++sn;
    if (g.reg && (k == 5 || k == TW - 1)) record_group<T, NF, F0, NG>(g, fn, k - 5, x, y, H);
    if (kk >= 6) {
      const int i = k - 6;  // interior cell along z
      const int ai = (i - k0) * ACC_PLANE + y * ACC_PITCH + x;
      double src[4] = {0.0, 0.0, 0.0, 0.0};
      const bool rot = F0 == 0 && g.omega != 0.0;
      if (rot) {
        const double dx = 1.0 / (double)(SUB * li.blocks);
        const double rx = ((double)(SUB * li.ix + x) + 0.5) * dx - 0.5;
        const double ry = ((double)(SUB * li.iy + y) + 0.5) * dx - 0.5;
        const double rho = (double)st[0].qy, sx = (double)st[1].qy, sy = (double)st[2].qy;
        const double om2 = g.omega * g.omega, tw = 2.0 * g.omega;
        src[0] = tw * sy + rho * om2 * rx;
        src[1] = rho * om2 * ry - tw * sx;
        src[3] = om2 * (sx * rx + sy * ry);
      }
      T cv[NF_CORE];
#pragma unroll
      for (int f = 0; f < NG; ++f) {
        const int fg = F0 + f;
        const double sum = acc[fg * ACC_HALF + ai] + ((double)H[f] - Hprev[f]);
        const T o = finish_cell<T>(s, (size_t)fg * fs, leaf_at + i * 64, st[f].qy, u0v[f], sum,
                                   rot && fg >= 1 && fg <= 4,
                                   fg >= 1 && fg <= 4 ? src[fg - 1] : 0.0, dt, inv_dx);
        if (F0 == 0 && f < NF_CORE) cv[f] = o;
        if constexpr (MODE == STEP_RESTRICT) {
          if (lnode >= 0)
            restrict_out<T, ACC_PLANE>(s, &acc[fg * ACC_HALF + ai], lnode, fg, x, y, i, o);
        }
      }
      if constexpr (MODE == STEP_CFL && F0 == 0)
        cflmin = fmin(cflmin, cfl_quantity<T>(g, cv, 1.0 / inv_dx));
    }
#pragma unroll
    for (int f = 0; f < NG; ++f) Hprev[f] = (double)H[f];
  }
}

// W = waves per SIMD the register budget allows (1: up to 512 VGPRs, 2: 256);
// MODE as for k_step.
template <typename T, int NF, int W, int MODE>
__global__ void __launch_bounds__(128, W) k_step2(StepArgs s) {
  static_assert(NF > NF_CORE, "the second wavefront needs passive species");
  __shared__ __align__(16) double acc[NF * ACC_HALF];
  __shared__ SpeedSlot<T> spd[2];
  const GridArgs& g = s.g;
  const int leaf = s.leaf_base + leaf_of_block(blockIdx.x, g.n_leaves, s.remap);
  if (leaf >= g.n_leaves) return;  // uniform over the workgroup
  // the role of each wavefront alternates with the workgroup, so that the
  // SIMDs the hardware deals consecutive wavefronts to carry core and
  // species work in equal shares
  const int wave = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) ^ (blockIdx.x & 1));
  const int lane = threadIdx.x & 63;

  LeafInfo li;
  li.leaf = leaf;
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  li.ix = c4.y;
  li.iy = c4.z;
  li.iz = c4.w;
  li.blocks = g.base << c4.x;
  const uint8_t* kd = g.kind + 27 * leaf;
  const int32_t* nb = g.nbr + 27 * leaf;
  const bool xlane = lane < 32;
  FaceNbr fxy, fz;
  fxy.klo = xlane ? (int)kd[12] : (int)kd[10];
  fxy.ilo = xlane ? nb[12] : nb[10];
  fxy.khi = xlane ? (int)kd[14] : (int)kd[16];
  fxy.ihi = xlane ? nb[14] : nb[16];
  fz.klo = kd[4];
  fz.ilo = nb[4];
  fz.khi = kd[22];
  fz.ihi = nb[22];
  fxy.rlo = fxy.rhi = fxy.flo = fxy.fhi = -1;
  fz.rlo = fz.rhi = fz.flo = fz.fhi = -1;
  if (g.reg) {
    const int32_t* fsl = g.face_slot + 6 * leaf;
    const int32_t* fin = g.fine_slot + 6 * leaf;
    fxy.rlo = xlane ? fsl[0] : fsl[2];
    fxy.rhi = xlane ? fsl[1] : fsl[3];
    fxy.flo = xlane ? fin[0] : fin[2];
    fxy.fhi = xlane ? fin[1] : fin[3];
    fz.rlo = fsl[4];
    fz.rhi = fsl[5];
    fz.flo = fin[4];
    fz.fhi = fin[5];
  }
  const double dt = *s.dt;
  const double inv_dx = (double)(SUB * li.blocks);
  Phys<T> ph;
  ph.gamma = (T)g.gamma;
  ph.gm1 = (T)(g.gamma - 1.0);
  ph.eta1 = (T)g.eta1;

  bool bad = false;
  double cflmin = INFINITY;
  const int lnode = MODE == STEP_RESTRICT ? g.leaf_node[leaf] : -1;
  int sn = 0;  // stream steps taken: selects the hand-off slot
  constexpr int NS = NF - NF_CORE;
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    if (wave == 0)
      phase_xy_group<T, NF, 0, NF_CORE>(s, ph, li, fxy, acc, spd, sn, h, lane, bad);
    else
      phase_xy_group<T, NF, NF_CORE, NS>(s, ph, li, fxy, acc, spd, sn, h, lane, bad);
    wave_lds_sync();
    if (wave == 0)
      phase_z_group<T, NF, 0, NF_CORE, MODE>(s, ph, li, fz, acc, spd, sn, h, lane, dt, inv_dx,
                                            bad, cflmin, lnode);
    else
      phase_z_group<T, NF, NF_CORE, NS, MODE>(s, ph, li, fz, acc, spd, sn, h, lane, dt, inv_dx,
                                             bad, cflmin, lnode);
    wave_lds_sync();
  }
  if constexpr (MODE == STEP_CFL) {
    if (wave == 0) atomic_min_positive(s.dt_next, cflmin, lane);
  }
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
}

// Launch shape of the fused substep: waves per SIMD (register budget) and
// wavefronts per leaf (1: k_step; 2: k_step2, species on the second).
struct StepShape {
  int waves_per_simd;
  int waves_per_leaf;
};

template <typename T, int NF, int MODE>
inline hipError_t launch_step_nf(const StepArgs& a, int blocks, StepShape sh, hipStream_t st) {
  if constexpr (NF > NF_CORE) {
    if (sh.waves_per_leaf == 2) {
      if (sh.waves_per_simd == 2)
        hipLaunchKernelGGL((k_step2<T, NF, 2, MODE>), dim3(blocks), dim3(128), 0, st, a);
      else
        hipLaunchKernelGGL((k_step2<T, NF, 1, MODE>), dim3(blocks), dim3(128), 0, st, a);
      return hipGetLastError();
    }
  }
  if (sh.waves_per_simd == 2)
    hipLaunchKernelGGL((k_step<T, NF, 2, MODE>), dim3(blocks), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_step<T, NF, 1, MODE>), dim3(blocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

// Launch of the fused substep for any field count in one MODE.
template <typename T, int MODE>
inline hipError_t launch_step_t(const StepArgs& a, int blocks, StepShape sh, hipStream_t st) {
  switch (a.g.nf) {
    case 6: return launch_step_nf<T, 6, MODE>(a, blocks, sh, st);
    case 7: return launch_step_nf<T, 7, MODE>(a, blocks, sh, st);
    case 8: return launch_step_nf<T, 8, MODE>(a, blocks, sh, st);
    case 9: return launch_step_nf<T, 9, MODE>(a, blocks, sh, st);
    case 10: return launch_step_nf<T, 10, MODE>(a, blocks, sh, st);
    case 11: return launch_step_nf<T, 11, MODE>(a, blocks, sh, st);
    case 12: return launch_step_nf<T, 12, MODE>(a, blocks, sh, st);
    case 13: return launch_step_nf<T, 13, MODE>(a, blocks, sh, st);
    case 14: return launch_step_nf<T, 14, MODE>(a, blocks, sh, st);
    case 15: return launch_step_nf<T, 15, MODE>(a, blocks, sh, st);
    case 16: return launch_step_nf<T, 16, MODE>(a, blocks, sh, st);
    default: return hipErrorInvalidValue;
  }
}

// One translation unit each.
hipError_t launch_step_f64(const StepArgs& a, int blocks, StepShape sh, hipStream_t st);
hipError_t launch_step_f32(const StepArgs& a, int blocks, StepShape sh, hipStream_t st);
hipError_t launch_step_f64_cfl(const StepArgs& a, int blocks, StepShape sh, hipStream_t st);
hipError_t launch_step_f32_cfl(const StepArgs& a, int blocks, StepShape sh, hipStream_t st);
hipError_t launch_step_f64_restrict(const StepArgs& a, int blocks, StepShape sh, hipStream_t st);
hipError_t launch_step_f32_restrict(const StepArgs& a, int blocks, StepShape sh, hipStream_t st);
hipError_t launch_step3d(const StepArgs& a, int dtype, int blocks, const void* G, int wg,
                         hipStream_t st);

}  // namespace octohydro
