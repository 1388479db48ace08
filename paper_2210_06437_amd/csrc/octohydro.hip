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
// A buffer offset past the end of every array the kernels address (array
// sizes are bounded below it on the host): a buffer load there returns 0
// without touching memory.
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
__device__ __noinline__ double tau_energy(double tau, double gamma) { return pow(tau, gamma); }
__device__ __noinline__ float tau_energy(float tau, float gamma) { return powf(tau, gamma); }

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
  uint32_t ouk;  // offset into the stage input, OFF_NONE on a refined side
  uint32_t orn;  // offset into the node copies, OFF_NONE elsewhere
  bool ref;      // this lane's value comes from a node copy
  bool any_ref;  // some lane of the wave reads a node copy (wave-uniform)
};

__device__ __forceinline__ Src pencil_src(const Pencil& p, int k) {
  Src s;
  if (k >= GH && k < GH + SUB) {
    s.o = s.ouk = p.off + (uint32_t)(k - GH) * p.sd;
    s.orn = OFF_NONE;
    s.ref = s.any_ref = false;
    return s;
  }
  s.o = k == 0 ? p.gofs[0] : k == 1 ? p.gofs[1] : k == 2 ? p.gofs[2]
      : k == 11 ? p.gofs[3] : k == 12 ? p.gofs[4] : p.gofs[5];
  s.ref = k < GH ? p.ref_lo : p.ref_hi;
  s.any_ref = k < GH ? p.any_lo : p.any_hi;
  s.ouk = s.ref ? OFF_NONE : s.o;
  s.orn = s.ref ? s.o : OFF_NONE;
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

// The two arrays stream values come from: the stage input (all interior and
// same-level or coarser ghosts) and the restricted node copies (ghosts on a
// refined side), each with its field stride in bytes.
struct Sources {
  Rsrc uk, rn;
  uint32_t uk_fs, rn_fs;
};

// The values of a stream position in all NF fields.  Where some lane of the
// wave reads a node copy, every lane loads from both arrays, one load with
// an offset past the end (which reads 0 without a memory access), and keeps
// its own: no divergent branch.  The test is made once per position, not
// once per field.
template <typename T, int NF>
__device__ __forceinline__ void load_position(const Sources& S, const Src& s, T (&q)[NF]) {
  if (s.any_ref) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const T a = bload(T(), FieldView{S.uk, f * S.uk_fs}, s.ouk);
      const T b = bload(T(), FieldView{S.rn, f * S.rn_fs}, s.orn);
      q[f] = s.ref ? b : a;
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
__device__ __forceinline__ void finish_cell(const StepArgs& s, size_t fbase, uint32_t cell, T uk,
                                            T u0, double sum, bool has_src, double src,
                                            double dt, double inv_dx) {
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
    OCTOHYDRO_FENCE();
  }
  core_flux(ph, d, core_L, core_R, Hc, vL, vR, ha, bad);
#pragma unroll
  for (int f = 0; f < NF_CORE; ++f) H[f] = Hc[f];
#pragma unroll
  for (int f = NF_CORE; f < NF; ++f) {
    OCTOHYDRO_FENCE();
    T ul, ur;
    ppm_push(st[f], qn[f], 5, ul, ur);
    H[f] = T(0.5) * (ul * vL + ur * vR) - ha * (ur - ul);
  }
}

// Phase XY of half h: lanes 0-31 stream x-pencils, lanes 32-63 y-pencils of
// the planes z in [4h, 4h+4).  Each cell receives dHx from one lane and dHy
// from another, both as LDS atomic adds (ds_add_f64, which rounds as binary64
// addition does) into an accumulator cleared to -0.0: -0.0 is the identity of
// binary64 addition (it keeps the sign of a zero term) and a sum of two terms
// does not depend on their order, so the accumulator holds exactly dHx + dHy
// whichever lane gets there first, with no branch on the lane.
template <typename T, int NF>
__device__ __forceinline__ void phase_xy(const StepArgs& s, const Phys<T>& ph, const LeafInfo& li,
                                         const FaceNbr& fn, double* __restrict__ acc, int h,
                                         int lane, bool& bad) {
  const GridArgs& g = s.g;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const Rsrc Uk = state_rsrc(s.Uk, (uint32_t)(g.nf * fs * sizeof(T)));
  const uint32_t fs_b = (uint32_t)(fs * sizeof(T));
  const uint32_t rn_fs = (uint32_t)((size_t)g.n_nodes * CELLS * sizeof(T));
  const Sources S{Uk, state_rsrc(g.rstate, g.rstate ? (uint32_t)g.nf * rn_fs : 0u), fs_b, rn_fs};
  const int d = lane >> 5;
  const int a = lane & 7;
  const int zz = (lane >> 3) & 3;
  const Pencil p = make_pencil<T>(g, li, d, a, 4 * h + zz, fn);
  const int acc_off = d == 0 ? zz * ACC_PLANE + a * ACC_PITCH : zz * ACC_PLANE + a;
  const int acc_step = d == 0 ? 1 : ACC_PITCH;

  for (int j = lane; j < NF * ACC_HALF / 2; j += 64)
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
        __hip_atomic_fetch_add(&acc[f * ACC_HALF + ai], dH[f], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) Hprev[f] = (double)H[f];
  }
}

// Phase Z of half h: lane (x, y) streams its z-pencil over stream positions
// [4h, 4h+10), which yields the z-faces of cells z in [4h, 4h+4), adds dHz
// to the accumulator and finishes those cells.
template <typename T, int NF>
__device__ __forceinline__ void phase_z(const StepArgs& s, const Phys<T>& ph, const LeafInfo& li,
                                        const FaceNbr& fn, const double* __restrict__ acc, int h,
                                        int lane, double dt, double inv_dx, bool& bad) {
  const GridArgs& g = s.g;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const Rsrc Uk = state_rsrc(s.Uk, (uint32_t)(g.nf * fs * sizeof(T)));
  const uint32_t fs_b = (uint32_t)(fs * sizeof(T));
  const uint32_t rn_fs = (uint32_t)((size_t)g.n_nodes * CELLS * sizeof(T));
  const Sources S{Uk, state_rsrc(g.rstate, g.rstate ? (uint32_t)g.nf * rn_fs : 0u), fs_b, rn_fs};
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
#pragma unroll 1
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
      for (int f = 0; f < NF; ++f) u0v[f] = bload(T(), FieldView{U0, f * fs_b}, cell_b);
    }
    T H[NF];
    stream_step<T, NF>(ph, 2, st, qn, H, bad);
    if (g.reg && (k == 5 || k == TW - 1)) record_face<T, NF>(g, fn, k - 5, x, y, H);
    if (kk >= 6) {
      const int i = k - 6;  // interior cell along z
      const int ai = (i - k0) * ACC_PLANE + y * ACC_PITCH + x;
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
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double sum = acc[f * ACC_HALF + ai] + ((double)H[f] - Hprev[f]);
        finish_cell<T>(s, (size_t)f * fs, leaf_at + i * 64, st[f].qy, u0v[f], sum,
                       rot && f >= 1 && f <= 4, f >= 1 && f <= 4 ? src[f - 1] : 0.0, dt, inv_dx);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) Hprev[f] = (double)H[f];
  }
}

// W = register budget: W waves per SIMD (1: up to 512 VGPRs, 2: up to 256).
template <typename T, int NF, int W>
__global__ void __launch_bounds__(64, W) k_step(StepArgs s) {
  __shared__ __align__(16) double acc[NF * ACC_HALF];
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
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    phase_xy<T, NF>(s, ph, li, fxy, acc, h, lane, bad);
    wave_lds_sync();
    phase_z<T, NF>(s, ph, li, fz, acc, h, lane, dt, inv_dx, bad);
    wave_lds_sync();
  }
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
}

// ---------------------------------------------------------------------------
// Full three-dimensional reconstruction with face quadrature (Sec. V-B-1: the
// reconstruct kernel does a full 3D reconstruction, the flux kernel integrates
// each face's flux by quadrature).
//
// Each cell gets values at its 26 face, edge and corner points: the point
// t + p/2 (p in {-1,0,1}^3, not 0) comes from the PPM of the axis scheme on
// the 5 cells t + m e, m = -2..2, with e = p or -p (first non-zero component
// positive): the right end of the cell's parabola when e = p, else the left
// end.  A face normal to D gets the Kurganov-Tadmor flux at its 9 points
// (pu, pv) in {-1,0,1}^2 (u < v the other two axes) -- left state from the
// left cell at (+1, pu, pv)/2, right state from the right cell at
// (-1, pu, pv)/2 -- combined by the tensor Simpson rule
//   ((corners + 4 edges) + 16 centre) / 36,
//   corners = (H(-1,-1) + H(1,1)) + (H(1,-1) + H(-1,1)),
//   edges   = (H(0,-1) + H(0,1)) + (H(-1,0) + H(1,0)).
//
// Ghost cells come from tiles materialised by k_fill (all 26 regions: the
// diagonal lines reach edge and corner ghosts).
// ---------------------------------------------------------------------------

// One end of the PPM parabola of the cell at t along a line of tile stride s.
template <typename T>
__device__ __forceinline__ T line_end(const T* __restrict__ t, int s, bool right) {
  const T q0 = t[-2 * s], q1 = t[-s], q2 = t[0], q3 = t[s], q4 = t[2 * s];
  const T dm1 = limited_slope(q0, q1, q2);
  const T dm2 = limited_slope(q1, q2, q3);
  const T dm3 = limited_slope(q2, q3, q4);
  T l = T(0.5) * (q1 + q2) - (dm2 - dm1) * T(1.0 / 6.0);
  T r = T(0.5) * (q2 + q3) - (dm3 - dm2) * T(1.0 / 6.0);
  monotonise(q2, l, r);
  return right ? r : l;
}

// Tile stride of the line that gives point p, and whether p is its right end.
struct PointLine {
  int s;
  bool right;
};

__device__ __forceinline__ constexpr PointLine point_line(int px, int py, int pz) {
  return PointLine{((px != 0 ? px : (py != 0 ? py : pz)) > 0 ? 1 : -1) *
                       (px + TW * py + TW * TW * pz),
                   (px != 0 ? px : (py != 0 ? py : pz)) > 0};
}

// Point offset components of face point (pu, pv) on side sd (+1 left cell,
// -1 right cell) of a face normal to D.
template <int D>
__device__ __forceinline__ constexpr PointLine face_point(int sd, int pu, int pv) {
  return D == 0 ? point_line(sd, pu, pv) : (D == 1 ? point_line(pu, sd, pv)
                                                   : point_line(pu, pv, sd));
}

// Simpson combination of the 9 point values of one field, points in the
// order (-1,-1), (1,1), (1,-1), (-1,1), (0,-1), (0,1), (-1,0), (1,0), (0,0).
template <typename T>
__device__ __forceinline__ T simpson9(const T (&h)[9]) {
  const T corners = (h[0] + h[1]) + (h[2] + h[3]);
  const T edges = (h[4] + h[5]) + (h[6] + h[7]);
  return ((corners + T(4) * edges) + T(16) * h[8]) / T(36);
}

// Flux of all fields through the face between tile cells tl and tl + stride
// of D (Gt: field 0's tile of the leaf, field stride fsG).  The core fields'
// end values at all 9 points are read first (their loads are independent, so
// many are in flight at once) and give the points' Kurganov-Tadmor fluxes,
// velocities and signal speeds; each passive field then uses those speeds.
template <typename T, int NF, int D>
__device__ __forceinline__ void face_flux_3d(const Phys<T>& ph, const T* __restrict__ Gt,
                                             size_t fsG, int tl, T (&H)[NF], bool& bad) {
  constexpr int SD = D == 0 ? 1 : (D == 1 ? TW : TW * TW);
  constexpr int PU[9] = {-1, 1, 1, -1, 0, 0, -1, 1, 0};
  constexpr int PV[9] = {-1, 1, -1, 1, -1, 1, 0, 0, 0};
  const int tr = tl + SD;
  T hc[NF_CORE][9], vl[9], vr[9], ha[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const PointLine pl = face_point<D>(1, PU[q], PV[q]);
    const PointLine pr = face_point<D>(-1, PU[q], PV[q]);
    T UL[NF_CORE], UR[NF_CORE], Hc[NF_CORE];
#pragma unroll
    for (int f = 0; f < NF_CORE; ++f) {
      UL[f] = line_end(Gt + f * fsG + tl, pl.s, pl.right);
      UR[f] = line_end(Gt + f * fsG + tr, pr.s, pr.right);
    }
    core_flux(ph, D, UL, UR, Hc, vl[q], vr[q], ha[q], bad);
#pragma unroll
    for (int f = 0; f < NF_CORE; ++f) hc[f][q] = Hc[f];
  }
#pragma unroll
  for (int f = 0; f < NF_CORE; ++f) H[f] = simpson9(hc[f]);
#pragma unroll
  for (int f = NF_CORE; f < NF; ++f) {
    T h[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const PointLine pl = face_point<D>(1, PU[q], PV[q]);
      const PointLine pr = face_point<D>(-1, PU[q], PV[q]);
      const T ul = line_end(Gt + f * fsG + tl, pl.s, pl.right);
      const T ur = line_end(Gt + f * fsG + tr, pr.s, pr.right);
      h[q] = T(0.5) * (ul * vl[q] + ur * vr[q]) - ha[q] * (ur - ul);
    }
    H[f] = simpson9(h);
  }
}

// Face-neighbour register slots of the faces normal to axis D.
__device__ __forceinline__ FaceNbr face_slots_3d(const GridArgs& g, int leaf, int D) {
  FaceNbr fn;
  fn.klo = fn.ilo = fn.khi = fn.ihi = 0;
  fn.rlo = fn.rhi = fn.flo = fn.fhi = -1;
  if (g.reg) {
    fn.rlo = g.face_slot[6 * leaf + 2 * D];
    fn.rhi = g.face_slot[6 * leaf + 2 * D + 1];
    fn.flo = g.fine_slot[6 * leaf + 2 * D];
    fn.fhi = g.fine_slot[6 * leaf + 2 * D + 1];
  }
  return fn;
}

// Tile index of leaf cell (x, y, z); -1 and 8 name the ghost layers.
__device__ __forceinline__ constexpr int tile_at(int x, int y, int z) {
  return (x + GH) + (y + GH) * TW + (z + GH) * TW * TW;
}

// One wave per leaf sweeps the z-planes; lane (x, y) owns cell (x, y, z) of
// the current plane.  A face's flux depends on no other face, so each plane
// costs three face evaluations per lane, each of them a wave-wide load of
// consecutive x-cells: the cell's low x-face, its low y-face and its high
// z-face.  The high x-face (y-face) of a cell is the low face of lane x+1
// (y+1), taken by a lane shuffle; for x = 7 (y = 7) it is face 8 of the row
// (column), which a first pass evaluates for the whole leaf and keeps in LDS.
// The low z-face is the high z-face of the plane before, kept in registers
// (z-face 0 comes from the first pass).  The differences are summed
// ((x + y) + z) in binary64 and the cell is finished as k_step does.
template <typename T, int NF>
__global__ void __launch_bounds__(64) k_step3d(StepArgs s, const T* __restrict__ G) {
  __shared__ double hx8[NF * 64];  // x-face 8 of row (y, z), at z * 8 + y
  __shared__ double hy8[NF * 64];  // y-face 8 of column (x, z), at z * 8 + x
  const GridArgs& g = s.g;
  const int leaf = s.leaf_base + blockIdx.x;
  if (leaf >= g.n_leaves) return;
  const int lane = threadIdx.x;
  LeafInfo li;
  li.leaf = leaf;
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  li.ix = c4.y;
  li.iy = c4.z;
  li.iz = c4.w;
  li.blocks = g.base << c4.x;
  const double dt = *s.dt;
  const double inv_dx = (double)(SUB * li.blocks);
  Phys<T> ph;
  ph.gamma = (T)g.gamma;
  ph.gm1 = (T)(g.gamma - 1.0);
  ph.eta1 = (T)g.eta1;
  const size_t fsG = (size_t)g.n_leaves * TILE;
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const T* __restrict__ Gt = G + (size_t)leaf * TILE;
  const FaceNbr fx = face_slots_3d(g, leaf, 0);
  const FaceNbr fy = face_slots_3d(g, leaf, 1);
  const FaceNbr fz = face_slots_3d(g, leaf, 2);
  const int x = lane & 7, y = lane >> 3;
  bool bad = false;
  const double dx = 1.0 / (double)(SUB * li.blocks);
  const double rx = ((double)(SUB * li.ix + x) + 0.5) * dx - 0.5;
  const double ry = ((double)(SUB * li.iy + y) + 0.5) * dx - 0.5;
  double Hz[NF];
  // z = -1 is the first pass: x-face 8 of row (a, b) and y-face 8 of column
  // (a, b), (a, b) = (lane & 7, lane >> 3), into LDS, and z-face 0 of the
  // lane's column into Hz.  Each later z evaluates the three faces of the
  // lane's cell and finishes it.
#pragma unroll 1
  for (int z = -1; z < SUB; ++z) {
    wave_lds_sync();  // the first pass's LDS values are read from z = 0 on
    const bool first = z < 0;
    T H[NF];
    double sxy[NF];
    face_flux_3d<T, NF, 0>(ph, Gt, fsG, first ? tile_at(SUB - 1, x, y) : tile_at(x - 1, y, z),
                           H, bad);
    if (first) {
      if (g.reg) record_face<T, NF>(g, fx, SUB, x, y, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) hx8[f * 64 + lane] = (double)H[f];
    } else {
      if (g.reg && x == 0) record_face<T, NF>(g, fx, 0, y, z, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double lo = (double)H[f];
        const double up = __shfl_down(lo, 1, 8);  // lane x+1: its low face
        const double hi = x == SUB - 1 ? hx8[f * 64 + z * 8 + y] : up;
        sxy[f] = hi - lo;
      }
    }
    face_flux_3d<T, NF, 1>(ph, Gt, fsG, first ? tile_at(x, SUB - 1, y) : tile_at(x, y - 1, z),
                           H, bad);
    if (first) {
      if (g.reg) record_face<T, NF>(g, fy, SUB, x, y, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) hy8[f * 64 + lane] = (double)H[f];
    } else {
      if (g.reg && y == 0) record_face<T, NF>(g, fy, 0, x, z, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double lo = (double)H[f];
        const double up = __shfl_down(lo, 8, 64);  // lane y+1: its low face
        const double hi = y == SUB - 1 ? hy8[f * 64 + z * 8 + x] : up;
        sxy[f] = sxy[f] + (hi - lo);
      }
    }
    face_flux_3d<T, NF, 2>(ph, Gt, fsG, tile_at(x, y, z), H, bad);
    if (first) {
      if (g.reg) record_face<T, NF>(g, fz, 0, x, y, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) Hz[f] = (double)H[f];
      continue;
    }
    if (g.reg && z == SUB - 1) record_face<T, NF>(g, fz, SUB, x, y, H);
    const T* __restrict__ ukc = Gt + tile_at(x, y, z);  // the cell's Uk
    double src[4] = {0.0, 0.0, 0.0, 0.0};
    const bool rot = g.omega != 0.0;
    if (rot) {
      const double rho = (double)ukc[0], sx = (double)ukc[fsG], sy = (double)ukc[2 * fsG];
      const double om2 = g.omega * g.omega, tw = 2.0 * g.omega;
      src[0] = tw * sy + rho * om2 * rx;
      src[1] = rho * om2 * ry - tw * sx;
      src[3] = om2 * (sx * rx + sy * ry);
    }
    const uint32_t at = (uint32_t)leaf * CELLS + z * 64 + lane;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double sum = sxy[f] + ((double)H[f] - Hz[f]);
      Hz[f] = (double)H[f];
      const T u0 = s.U0 ? static_cast<const T*>(s.U0)[(size_t)f * fs + at] : T(0);
      finish_cell<T>(s, (size_t)f * fs, at, ukc[f * fsG], u0, sum, rot && f >= 1 && f <= 4,
                     f >= 1 && f <= 4 ? src[f - 1] : 0.0, dt, inv_dx);
    }
  }
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
}

// ---------------------------------------------------------------------------
// Coarse-fine flux correction: one launch per face orientation o, one thread
// per (slot, field, coarse face cell); a coarse leaf has at most one slot per
// orientation, so no two threads of a launch touch the same value.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256)
    k_reflux(GridArgs g, T* __restrict__ Uout, const double* dt, double w, int o, int s0,
             int n_in_orient) {
  const int64_t total = (int64_t)n_in_orient * g.nf * 64;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int uv = (int)(idx & 63);
  const int64_t sf = idx >> 6;
  const int f = (int)(sf % g.nf);
  const int slot = s0 + (int)(sf / g.nf);
  const int u = uv & 7, v = uv >> 3;
  const int c = g.slot_leaf[slot];
  const double inv_dx = (double)(SUB * (g.base << g.coord[4 * c]));
  const double* r = g.reg + ((size_t)slot * g.nf + f) * REG_STRIDE;
  const double hc = r[u + 8 * v];
  const double* fr = r + REG_COARSE + 2 * u + 16 * (2 * v);
  const double havg = 0.25 * ((fr[0] + fr[1]) + (fr[16] + fr[17]));
  const double q = (havg - hc) * inv_dx;
  const double wdt = w * *dt;
  const int d = o >> 1, side = o & 1;
  int l[3];
  l[d] = side ? SUB - 1 : 0;
  l[d == 0 ? 1 : 0] = u;
  l[d == 2 ? 1 : 2] = v;
  T* out = Uout + ((size_t)f * g.n_leaves + c) * CELLS + l[2] * 64 + l[1] * 8 + l[0];
  const double val = (double)*out;
  *out = (T)(side ? val - wdt * q : val + wdt * q);
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
  if (gr->n_leaves > HYDRO_MAX_LEAVES)
    return fail(HYDRO_E_ARG, "%s: n_leaves %d exceeds %d (one field array must stay below 4 GiB)",
                fn, gr->n_leaves, HYDRO_MAX_LEAVES);
  if (gr->n_fields < NF_CORE || gr->n_fields > 16)
    return fail(HYDRO_E_ARG, "%s: n_fields must be in [6,16], got %d", fn, gr->n_fields);
  if (gr->dtype != HYDRO_F64 && gr->dtype != HYDRO_F32)
    return fail(HYDRO_E_ARG, "%s: unknown dtype %d", fn, gr->dtype);
  if (gr->base <= 0) return fail(HYDRO_E_ARG, "%s: base must be positive", fn);
  if (gr->reconstruction != HYDRO_RECON_AXIS && gr->reconstruction != HYDRO_RECON_3D)
    return fail(HYDRO_E_ARG, "%s: unknown reconstruction %d", fn, gr->reconstruction);
  if (!gr->leaf_coord_dev || !gr->nbr_dev || !gr->nbr_kind_dev)
    return fail(HYDRO_E_ARG, "%s: table pointers must be set", fn);
  if (gr->n_nodes > 0 && !gr->children_dev)
    return fail(HYDRO_E_ARG, "%s: children_dev is NULL but n_nodes > 0", fn);
  if (!(gr->gamma > 1.0)) return fail(HYDRO_E_ARG, "%s: gamma must exceed 1", fn);
  const uint64_t state_bytes = (uint64_t)gr->n_fields * (uint64_t)gr->n_leaves * CELLS *
                               (gr->dtype == HYDRO_F64 ? 8u : 4u);
  if (state_bytes > OFF_NONE)
    return fail(HYDRO_E_ARG, "%s: a state array of %llu bytes exceeds 4 GiB - 4 KiB", fn,
                (unsigned long long)state_bytes);
  if (gr->flux_reg_dev && gr->n_slots > 0) {
    if (!gr->face_slot_dev || !gr->fine_slot_dev || !gr->slot_leaf_dev)
      return fail(HYDRO_E_ARG, "%s: flux register set but its tables are not", fn);
    if (gr->orient_begin[0] != 0 || gr->orient_begin[6] != gr->n_slots)
      return fail(HYDRO_E_ARG, "%s: orient_begin does not span the slots", fn);
    for (int o = 0; o < 6; ++o)
      if (gr->orient_begin[o + 1] < gr->orient_begin[o])
        return fail(HYDRO_E_ARG, "%s: orient_begin is not ascending", fn);
  }
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
  const bool reflux = gr->flux_reg_dev != nullptr && gr->n_slots > 0;
  g.face_slot = reflux ? gr->face_slot_dev : nullptr;
  g.fine_slot = reflux ? gr->fine_slot_dev : nullptr;
  g.slot_leaf = reflux ? gr->slot_leaf_dev : nullptr;
  g.reg = reflux ? gr->flux_reg_dev : nullptr;
  g.omega = gr->omega;
  g.rstate = gr->n_nodes > 0 ? gr->node_state_dev : nullptr;
  return g;
}

// The flux-correction launches after a substep (nothing without tables).
static int reflux_launch(const hydro_grid* gr, const StepArgs& a, hipStream_t st) {
  if (!a.g.reg) return HYDRO_OK;
  const double w = a.U0 ? a.beta : 1.0;
  for (int o = 0; o < 6; ++o) {
    const int s0 = gr->orient_begin[o], n = gr->orient_begin[o + 1] - s0;
    if (n <= 0) continue;
    const int64_t total = (int64_t)n * a.g.nf * 64;
    const int blocks = (int)((total + 255) / 256);
    if (gr->dtype == HYDRO_F64)
      hipLaunchKernelGGL(k_reflux<double>, dim3(blocks), dim3(256), 0, st, a.g,
                         static_cast<double*>(a.Uout), a.dt, w, o, s0, n);
    else
      hipLaunchKernelGGL(k_reflux<float>, dim3(blocks), dim3(256), 0, st, a.g,
                         static_cast<float*>(a.Uout), a.dt, w, o, s0, n);
    HIP_TRY(hipGetLastError());
  }
  return HYDRO_OK;
}

static int grid_blocks(int64_t work, int threads, int cap) {
  int64_t b = (work + threads - 1) / threads;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

// Ghosted 14^3 tiles of U into G (all 26 ghost regions).
static int fill_launch(const hydro_grid* gr, const void* U, void* G, hipStream_t st) {
  const GridArgs g = grid_args(gr);
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

// The restricted node copies of a substep's input state (nothing without
// refined nodes).
static int restrict_launch(const hydro_grid* gr, const void* Uk, hipStream_t st) {
  if (gr->n_nodes <= 0) return HYDRO_OK;
  const GridArgs g = grid_args(gr);
  const dim3 grid(g.n_nodes, g.nf);
  if (gr->dtype == HYDRO_F64)
    hipLaunchKernelGGL(k_restrict<double>, grid, dim3(CELLS), 0, st, g,
                       static_cast<const double*>(Uk), static_cast<double*>(gr->node_state_dev));
  else
    hipLaunchKernelGGL(k_restrict<float>, grid, dim3(CELLS), 0, st, g,
                       static_cast<const float*>(Uk), static_cast<float*>(gr->node_state_dev));
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

// Launch options per (dtype, n_fields), set by hydro_set_option (the
// autotuner's choices) and read at launch time.
struct Options {
  int waves_per_simd = 1;
  int xcd_remap = 1;
};
static Options g_opts[2][17];
static std::mutex g_opts_mu;

static Options get_options(int dtype, int nf) {
  std::lock_guard<std::mutex> lk(g_opts_mu);
  return g_opts[dtype][nf];
}

template <typename T, int NF>
static hipError_t launch_step_nf(const StepArgs& a, int blocks, int waves, hipStream_t st) {
  if (waves == 2)
    hipLaunchKernelGGL((k_step<T, NF, 2>), dim3(blocks), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_step<T, NF, 1>), dim3(blocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_step_t(const StepArgs& a, int blocks, int waves, hipStream_t st) {
  switch (a.g.nf) {
    case 6: return launch_step_nf<T, 6>(a, blocks, waves, st);
    case 7: return launch_step_nf<T, 7>(a, blocks, waves, st);
    case 8: return launch_step_nf<T, 8>(a, blocks, waves, st);
    case 9: return launch_step_nf<T, 9>(a, blocks, waves, st);
    case 10: return launch_step_nf<T, 10>(a, blocks, waves, st);
    case 11: return launch_step_nf<T, 11>(a, blocks, waves, st);
    case 12: return launch_step_nf<T, 12>(a, blocks, waves, st);
    case 13: return launch_step_nf<T, 13>(a, blocks, waves, st);
    case 14: return launch_step_nf<T, 14>(a, blocks, waves, st);
    case 15: return launch_step_nf<T, 15>(a, blocks, waves, st);
    case 16: return launch_step_nf<T, 16>(a, blocks, waves, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_step3d_t(const StepArgs& a, int blocks, const T* G, hipStream_t st) {
  switch (a.g.nf) {
#define OCTOHYDRO_CASE3D(n) \
  case n: hipLaunchKernelGGL((k_step3d<T, n>), dim3(blocks), dim3(64), 0, st, a, G); break;
    OCTOHYDRO_CASE3D(6) OCTOHYDRO_CASE3D(7) OCTOHYDRO_CASE3D(8) OCTOHYDRO_CASE3D(9)
    OCTOHYDRO_CASE3D(10) OCTOHYDRO_CASE3D(11) OCTOHYDRO_CASE3D(12) OCTOHYDRO_CASE3D(13)
    OCTOHYDRO_CASE3D(14) OCTOHYDRO_CASE3D(15) OCTOHYDRO_CASE3D(16)
#undef OCTOHYDRO_CASE3D
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_step3d(const StepArgs& a, int dtype, int blocks, const void* G,
                                hipStream_t st) {
  return dtype == HYDRO_F64 ? launch_step3d_t<double>(a, blocks, static_cast<const double*>(G), st)
                            : launch_step3d_t<float>(a, blocks, static_cast<const float*>(G), st);
}

static hipError_t launch_step(StepArgs a, int dtype, int blocks, hipStream_t st) {
  const Options o = get_options(dtype, a.g.nf);
  if (a.remap) a.remap = o.xcd_remap;
  return dtype == HYDRO_F64 ? launch_step_t<double>(a, blocks, o.waves_per_simd, st)
                            : launch_step_t<float>(a, blocks, o.waves_per_simd, st);
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
  if (!Uk || !Uout || !dt) return fail(HYDRO_E_ARG, "%s: Uk, Uout and dt must be set", fn);
  if (Uout == Uk || (U0 && Uout == U0))
    return fail(HYDRO_E_ARG, "%s: Uout may not alias an input", fn);
  if (flags & ~(HYDRO_FLAG_VALIDATE | HYDRO_FLAG_NODES_READY))
    return fail(HYDRO_E_ARG, "%s: unknown flags", fn);
  if (gr->reconstruction == HYDRO_RECON_3D) {
    if (!gr->ghost_tile_dev)
      return fail(HYDRO_E_ARG, "%s: ghost_tile_dev is NULL but reconstruction is 3D", fn);
    if (gr->ghost_tile_dev == Uk || gr->ghost_tile_dev == Uout || (U0 && gr->ghost_tile_dev == U0))
      return fail(HYDRO_E_ARG, "%s: ghost_tile_dev may not alias a state array", fn);
  } else if (gr->n_nodes > 0) {
    if (!gr->node_state_dev)
      return fail(HYDRO_E_ARG, "%s: node_state_dev is NULL but n_nodes > 0", fn);
    const uint64_t node_bytes = (uint64_t)gr->n_fields * (uint64_t)gr->n_nodes * CELLS *
                                (gr->dtype == HYDRO_F64 ? 8u : 4u);
    if (node_bytes > OFF_NONE)
      return fail(HYDRO_E_ARG, "%s: node_state of %llu bytes exceeds 4 GiB - 4 KiB", fn,
                  (unsigned long long)node_bytes);
  }
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

// One substep on `st`: the pre-pass of the reconstruction (restricted node
// copies, or the materialised tiles of the 3D mode), the step kernel over
// `blocks` leaves from a.leaf_base, and nothing else.
static int substep_kernels(const hydro_grid* gr, const StepArgs& a, int blocks, bool pre,
                           hipStream_t st) {
  int rc;
  if (gr->reconstruction == HYDRO_RECON_3D) {
    if (pre && (rc = fill_launch(gr, a.Uk, gr->ghost_tile_dev, st))) return rc;
    HIP_TRY(launch_step3d(a, gr->dtype, blocks, gr->ghost_tile_dev, st));
    return HYDRO_OK;
  }
  if (pre && (rc = restrict_launch(gr, a.Uk, st))) return rc;
  HIP_TRY(launch_step(a, gr->dtype, blocks, st));
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
  // every argument is checked before anything is queued
  StepArgs a;
  rc = step_common(gr, nullptr, Un, W1, dt, 1.0, 0, "hydro_rk3_step", a);
  if (rc) return rc;
  if (cfl > 0.0) {
    rc = cfl_launch(gr, Un, cfl, dt, st);
    if (rc) return rc;
  }
  if ((rc = substep_kernels(gr, a, gr->n_leaves, true, st))) return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
  a.U0 = Un;
  a.Uk = W1;
  a.Uout = W2;
  a.beta = 0.25;
  if ((rc = substep_kernels(gr, a, gr->n_leaves, true, st))) return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
  a.Uk = W2;
  a.Uout = Unext;
  a.beta = 2.0 / 3.0;
  if ((rc = substep_kernels(gr, a, gr->n_leaves, true, st))) return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
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

int hydro_set_option(int32_t dtype, int32_t n_fields, int32_t option, int32_t value) {
  clear_error();
  if ((dtype != HYDRO_F64 && dtype != HYDRO_F32) || n_fields < NF_CORE || n_fields > 16)
    return fail(HYDRO_E_ARG, "hydro_set_option: bad dtype %d or n_fields %d", dtype, n_fields);
  std::lock_guard<std::mutex> lk(g_opts_mu);
  Options& o = g_opts[dtype][n_fields];
  switch (option) {
    case HYDRO_OPT_WAVES_PER_SIMD:
      if (value != 1 && value != 2)
        return fail(HYDRO_E_ARG, "hydro_set_option: waves per SIMD must be 1 or 2");
      o.waves_per_simd = value;
      return HYDRO_OK;
    case HYDRO_OPT_XCD_REMAP:
      if (value != 0 && value != 1) return fail(HYDRO_E_ARG, "hydro_set_option: remap is 0 or 1");
      o.xcd_remap = value;
      return HYDRO_OK;
    default:
      return fail(HYDRO_E_ARG, "hydro_set_option: unknown option %d", option);
  }
}

int hydro_get_option(int32_t dtype, int32_t n_fields, int32_t option, int32_t* value) {
  clear_error();
  if ((dtype != HYDRO_F64 && dtype != HYDRO_F32) || n_fields < NF_CORE || n_fields > 16 || !value)
    return fail(HYDRO_E_ARG, "hydro_get_option: bad argument");
  const Options o = get_options(dtype, n_fields);
  if (option == HYDRO_OPT_WAVES_PER_SIMD) *value = o.waves_per_simd;
  else if (option == HYDRO_OPT_XCD_REMAP) *value = o.xcd_remap;
  else return fail(HYDRO_E_ARG, "hydro_get_option: unknown option %d", option);
  return HYDRO_OK;
}

const char* hydro_last_error(void) { return error_buffer(); }

int hydro_fill_ghosts(const hydro_grid* gr, const void* U, void* G, void* stream) {
  clear_error();
  int rc = check_grid(gr, "hydro_fill_ghosts");
  if (rc) return rc;
  if (!U || !G) return fail(HYDRO_E_ARG, "hydro_fill_ghosts: U and G must be set");
  if (U == G) return fail(HYDRO_E_ARG, "hydro_fill_ghosts: G may not alias U");
  return fill_launch(gr, U, G, static_cast<hipStream_t>(stream));
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
  if ((rc = substep_kernels(gr, a, gr->n_leaves, !(flags & HYDRO_FLAG_NODES_READY), st)))
    return rc;
  return reflux_launch(gr, a, st);
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
  // the pre-pass of the reconstruction runs once, on `stream`
  if (gr->reconstruction == HYDRO_RECON_3D) {
    if ((rc = fill_launch(gr, Uk, gr->ghost_tile_dev, st))) return rc;
  } else if ((rc = restrict_launch(gr, Uk, st))) {
    return rc;
  }
  // pool streams start after the work already queued on `stream`
  HIP_TRY(hipEventRecord(g_pool.events[0], st));
  for (int i = 0; i < n_streams; ++i) HIP_TRY(hipStreamWaitEvent(g_pool.streams[i], g_pool.events[0], 0));
  a.remap = 0;
  for (int leaf = 0; leaf < gr->n_leaves; ++leaf) {
    a.leaf_base = leaf;
    if ((rc = substep_kernels(gr, a, 1, false, g_pool.streams[leaf % n_streams]))) return rc;
  }
  for (int i = 0; i < n_streams; ++i) {
    HIP_TRY(hipEventRecord(g_pool.events[i], g_pool.streams[i]));
    HIP_TRY(hipStreamWaitEvent(st, g_pool.events[i], 0));
  }
  return reflux_launch(gr, a, st);
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
