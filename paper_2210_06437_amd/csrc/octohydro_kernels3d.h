// Device code of the full three-dimensional reconstruction with face
// quadrature (HYDRO_RECON_3D): the line reconstruction, the 9-point face flux
// and the k_step3d kernel with its launchers, on top of the method's shared
// device code in octohydro_kernels.h.  Included by the k_step3d units only.
#pragma once

#include "octohydro_kernels.h"

namespace octohydro {

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

// The PPM parabola of the cell at t along a line of tile stride s: its ends
// at t - s/2 (l) and t + s/2 (r).  Walking the line the other way (stride
// -s) gives the same two values with l and r exchanged, bit for bit: the
// limited slopes change sign exactly (or stay +0), the interface values and
// the monotonisation are symmetric in the two ends, and every sum involved
// is commutative.
template <typename T>
__device__ __forceinline__ void parabola(const T* __restrict__ t, int s, T& l, T& r) {
  const T q0 = t[-2 * s], q1 = t[-s], q2 = t[0], q3 = t[s], q4 = t[2 * s];
  const T dm1 = limited_slope(q0, q1, q2);
  const T dm2 = limited_slope(q1, q2, q3);
  const T dm3 = limited_slope(q2, q3, q4);
  l = T(0.5) * (q1 + q2) - (dm2 - dm1) * T(1.0 / 6.0);
  r = T(0.5) * (q2 + q3) - (dm3 - dm2) * T(1.0 / 6.0);
  monotonise(q2, l, r);
}

// One end of the PPM parabola of the cell at t along a line of tile stride s.
template <typename T>
__device__ __forceinline__ T line_end(const T* __restrict__ t, int s, bool right) {
  T l, r;
  parabola(t, s, l, r);
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
    for (int f = 0; f < NF_CORE; ++f) {
      hc[f][q] = Hc[f];
      keep_order(hc[f][q]);
    }
    keep_order(vl[q]);
    keep_order(vr[q]);
    keep_order(ha[q]);
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
    keep_order(H[f]);
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

// One wave per leaf; lane (x, y) owns cell (x, y, z) of the current z-plane.
// A face's flux depends on no other face, so each plane costs three face
// evaluations per lane, each of them a wave-wide load of consecutive
// x-cells: the cell's low x-face, its low y-face and its high z-face.  The
// high x-face (y-face) of a cell is the low face of lane x+1 (y+1), taken by
// a lane shuffle; for x = 7 (y = 7) it is face 8 of the row (column), which
// a first pass evaluates for the whole leaf and keeps in LDS.  The low
// z-face is the high z-face of the plane before (z-face 0 comes from the
// first pass).  The differences are summed ((x + y) + z) in binary64 and the
// cell is finished as k_step does.
// binary64 runs at 1 wavefront per SIMD, two z-halves of three loops (one
// face orientation per loop): one face evaluation nearly fills the 512
// registers, and three of them in one loop body spilled 333 VGPRs to memory
// (80 in this layout; 110.7 vs 122.3 ms on the 65535-leaf case).  binary32
// runs at 2 wavefronts per SIMD (256 VGPRs; 63 ms vs 89 ms at 1) as one
// sweep with the three faces in one loop body, whose LDS (11 KB) keeps 8
// wavefronts per CU where the binary64 layout's 39 KB would allow 4.
template <typename T, int NF>
__global__ void __launch_bounds__(64, sizeof(T) == 4 ? 2 : 1)
    k_step3d(StepArgs s, const T* __restrict__ G) {
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
  if constexpr (sizeof(T) == 8) {
  // binary64: two z-halves, each in three loops over its 4 planes -- x-faces,
  // y-faces, z-faces -- so that one loop body holds one face evaluation.
  // Lane (x, y) keeps its cells' dHx + dHy in its own LDS slots (acc3) and
  // its low z-face flux in hz3.  The first half's loops start with a first
  // pass (zl = -1): x-face 8 of every row and y-face 8 of every column into
  // hx8/hy8, z-face 0 of the lane's column into hz3.
  __shared__ double acc3[NF * 256];  // dHx + dHy of the half's cells, [f][zl * 64 + lane]
  __shared__ double hz3[NF * 64];    // each lane's low z-face flux, [f][lane]
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int z0 = 4 * h, zs = h == 0 ? -1 : 0;
#pragma unroll 1
    for (int zl = zs; zl < 4; ++zl) {
      wave_lds_sync();
      const bool first = zl < 0;
      const int z = z0 + zl;
      T H[NF];
      face_flux_3d<T, NF, 0>(ph, Gt, fsG, first ? tile_at(SUB - 1, x, y) : tile_at(x - 1, y, z),
                             H, bad);
      if (first) {
        if (g.reg) record_face<T, NF>(g, fx, SUB, x, y, H);
#pragma unroll
        for (int f = 0; f < NF; ++f) hx8[f * 64 + lane] = (double)H[f];
        continue;
      }
      if (g.reg && x == 0) record_face<T, NF>(g, fx, 0, y, z, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double lo = (double)H[f];
        const double up = __shfl_down(lo, 1, 8);  // lane x+1: its low face
        const double hi = x == SUB - 1 ? hx8[f * 64 + z * 8 + y] : up;
        acc3[f * 256 + zl * 64 + lane] = hi - lo;
      }
    }
#pragma unroll 1
    for (int zl = zs; zl < 4; ++zl) {
      wave_lds_sync();
      const bool first = zl < 0;
      const int z = z0 + zl;
      T H[NF];
      face_flux_3d<T, NF, 1>(ph, Gt, fsG, first ? tile_at(x, SUB - 1, y) : tile_at(x, y - 1, z),
                             H, bad);
      if (first) {
        if (g.reg) record_face<T, NF>(g, fy, SUB, x, y, H);
#pragma unroll
        for (int f = 0; f < NF; ++f) hy8[f * 64 + lane] = (double)H[f];
        continue;
      }
      if (g.reg && y == 0) record_face<T, NF>(g, fy, 0, x, z, H);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double lo = (double)H[f];
        const double up = __shfl_down(lo, 8, 64);  // lane y+1: its low face
        const double hi = y == SUB - 1 ? hy8[f * 64 + z * 8 + x] : up;
        acc3[f * 256 + zl * 64 + lane] = acc3[f * 256 + zl * 64 + lane] + (hi - lo);
      }
    }
#pragma unroll 1
    for (int zl = zs; zl < 4; ++zl) {
      const int z = z0 + zl;
      T H[NF];
      face_flux_3d<T, NF, 2>(ph, Gt, fsG, tile_at(x, y, z), H, bad);
      if (zl < 0) {
        if (g.reg) record_face<T, NF>(g, fz, 0, x, y, H);
#pragma unroll
        for (int f = 0; f < NF; ++f) hz3[f * 64 + lane] = (double)H[f];
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
        const double sum = acc3[f * 256 + zl * 64 + lane] + ((double)H[f] - hz3[f * 64 + lane]);
        hz3[f * 64 + lane] = (double)H[f];
        const T u0 = s.U0 ? static_cast<const T*>(s.U0)[(size_t)f * fs + at] : T(0);
        finish_cell<T>(s, (size_t)f * fs, at, ukc[f * fsG], u0, sum, rot && f >= 1 && f <= 4,
                       f >= 1 && f <= 4 ? src[f - 1] : 0.0, dt, inv_dx);
      }
    }
  }
  } else {
  // binary32: one sweep over the planes, three faces per plane in one loop
  // body (at 2 wavefronts per SIMD the binary64 layout's 39 KB of LDS would
  // halve the occupancy)
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
  }
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
}

// Launch of k_step3d<T, NF>.  Its instantiations are explicit, spread over
// the k_step3d_<precision>_<fields>.hip units, which compile in parallel.
// ---------------------------------------------------------------------------
// The 3D step with one 256-thread workgroup (4 wavefronts) per leaf.  The
// leaf's face fluxes are 27 planes of 64 faces: the low x-faces of each of
// the 8 cell planes (lane (x, y): face between cells x - 1 and x), the low
// y-faces of each plane, the 9 planes of z-faces (between cell planes z - 1
// and z), and the leaf's high x- and y-faces (lane (y, z) and (x, z)).  The
// wavefronts take these face planes in turn (wavefront w evaluates planes
// w, w + 4, ...), keep every flux in LDS, and after one workgroup barrier
// all 256 threads finish the 512 cells.  One leaf per CU keeps the tile
// planes its wavefronts read at once in the XCD's L2.  Each face is the
// same face_flux_3d evaluation as in k_step3d and each cell the same sums
// ((dHx + dHy) + dHz), so the results are bit-identical to it.
// ---------------------------------------------------------------------------

// Face plane j of the task list: direction and plane, in an order that
// keeps the four wavefronts on neighbouring cell planes.
struct FacePlane {
  int d, p;  // d: 0 x, 1 y, 2 z; p: cell plane (x, y: 0..7, 8 = the high
             // boundary face) or z-face plane 0..8
};

__device__ __forceinline__ FacePlane face_plane(int j) {
  // x8, y8, then (z0), and per cell plane p: x p, y p, z p+1
  if (j == 0) return FacePlane{0, 8};
  if (j == 1) return FacePlane{1, 8};
  if (j == 2) return FacePlane{2, 0};
  const int k = j - 3, p = k / 3, r = k % 3;
  return r == 0 ? FacePlane{0, p} : (r == 1 ? FacePlane{1, p} : FacePlane{2, p + 1});
}
constexpr int FACE_PLANES = 27;

// LDS bytes of k_step3d_wg's flux store: 8 + 8 + 9 + 2 planes of 64 faces.
template <typename T, int NF>
constexpr size_t wg3d_lds_bytes() {
  return (size_t)FACE_PLANES * 64 * NF * sizeof(T);
}

// Cell finishing of the workgroup forms, after the barrier that follows the
// face fluxes: thread t of the 256 takes cells t and t + 256, each with the
// binary64 sums ((xhi - xlo) + (yhi - ylo)) + (zhi - zlo) from the flux
// store Hs (the layout of k_step3d_wg).
template <typename T, int NF, int P>
__device__ __forceinline__ void finish_leaf_3d(const StepArgs& s, const T (&Hs)[P][NF][64],
                                               int leaf, int4 c4) {
  const GridArgs& g = s.g;
  const int blocks = g.base << c4.x;
  const double dt = *s.dt;
  const double inv_dx = (double)(SUB * blocks);
  const double dx = 1.0 / (double)(SUB * blocks);
  const size_t fs = (size_t)g.n_leaves * CELLS;
  const T* __restrict__ Uk = static_cast<const T*>(s.Uk);
  const T* __restrict__ U0 = static_cast<const T*>(s.U0);
#pragma unroll 1
  for (int c = threadIdx.x; c < CELLS; c += 256) {
    const int x = c & 7, y = (c >> 3) & 7, z = c >> 6;
    const int xy = y * 8 + x;
    const uint32_t at = (uint32_t)leaf * CELLS + c;
    double src[4] = {0.0, 0.0, 0.0, 0.0};
    const bool rot = g.omega != 0.0;
    if (rot) {
      const double rx = ((double)(SUB * c4.y + x) + 0.5) * dx - 0.5;
      const double ry = ((double)(SUB * c4.z + y) + 0.5) * dx - 0.5;
      const double rho = (double)Uk[at], sx = (double)Uk[fs + at], sy = (double)Uk[2 * fs + at];
      const double om2 = g.omega * g.omega, tw = 2.0 * g.omega;
      src[0] = tw * sy + rho * om2 * rx;
      src[1] = rho * om2 * ry - tw * sx;
      src[3] = om2 * (sx * rx + sy * ry);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double xlo = (double)Hs[z][f][xy];
      const double xhi = (double)(x == SUB - 1 ? Hs[SUB][f][z * 8 + y] : Hs[z][f][xy + 1]);
      const double ylo = (double)Hs[9 + z][f][xy];
      const double yhi = (double)(y == SUB - 1 ? Hs[9 + SUB][f][z * 8 + x] : Hs[9 + z][f][xy + 8]);
      const double zlo = (double)Hs[18 + z][f][xy];
      const double zhi = (double)Hs[18 + z + 1][f][xy];
      const double sum = ((xhi - xlo) + (yhi - ylo)) + (zhi - zlo);
      const T u0 = U0 ? U0[(size_t)f * fs + at] : T(0);
      finish_cell<T>(s, (size_t)f * fs, at, Uk[(size_t)f * fs + at], u0, sum,
                     rot && f >= 1 && f <= 4, f >= 1 && f <= 4 ? src[f - 1] : 0.0, dt, inv_dx);
    }
  }
}

template <typename T, int NF>
__global__ void __launch_bounds__(256, 1) k_step3d_wg(StepArgs s, const T* __restrict__ G) {
  // fluxes, [plane][field][lane]: planes 0-7 low x-faces, 8 high x-faces,
  // 9-16 low y-faces, 17 high y-faces, 18-26 z-faces 0..8
  __shared__ T Hs[FACE_PLANES][NF][64];
  const GridArgs& g = s.g;
  const int leaf = s.leaf_base + blockIdx.x;
  if (leaf >= g.n_leaves) return;  // uniform over the workgroup
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  Phys<T> ph;
  ph.gamma = (T)g.gamma;
  ph.gm1 = (T)(g.gamma - 1.0);
  ph.eta1 = (T)g.eta1;
  const size_t fsG = (size_t)g.n_leaves * TILE;
  const T* __restrict__ Gt = G + (size_t)leaf * TILE;
  const int a = lane & 7, b = lane >> 3;
  bool bad = false;
#pragma unroll 1
  for (int j = wave; j < FACE_PLANES; j += 4) {
    const FacePlane fp = face_plane(j);
    T H[NF];
    int slot;
    if (fp.d == 0) {
      // lane (a, b) = (x, y) of a low face in plane p, or (y, z) of face 8
      const bool hi = fp.p == SUB;
      face_flux_3d<T, NF, 0>(ph, Gt, fsG, hi ? tile_at(SUB - 1, a, b) : tile_at(a - 1, b, fp.p),
                             H, bad);
      if (g.reg) {
        const FaceNbr fn = face_slots_3d(g, leaf, 0);
        if (hi) record_face<T, NF>(g, fn, SUB, a, b, H);
        else if (a == 0) record_face<T, NF>(g, fn, 0, b, fp.p, H);
      }
      slot = hi ? SUB : fp.p;
    } else if (fp.d == 1) {
      const bool hi = fp.p == SUB;
      face_flux_3d<T, NF, 1>(ph, Gt, fsG, hi ? tile_at(a, SUB - 1, b) : tile_at(a, b - 1, fp.p),
                             H, bad);
      if (g.reg) {
        const FaceNbr fn = face_slots_3d(g, leaf, 1);
        if (hi) record_face<T, NF>(g, fn, SUB, a, b, H);
        else if (b == 0) record_face<T, NF>(g, fn, 0, a, fp.p, H);
      }
      slot = 9 + (hi ? SUB : fp.p);
    } else {
      face_flux_3d<T, NF, 2>(ph, Gt, fsG, tile_at(a, b, fp.p - 1), H, bad);
      if (g.reg && (fp.p == 0 || fp.p == SUB))
        record_face<T, NF>(g, face_slots_3d(g, leaf, 2), fp.p, a, b, H);
      slot = 18 + fp.p;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) Hs[slot][f][lane] = H[f];
  }
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
  __syncthreads();
  finish_leaf_3d<T, NF, FACE_PLANES>(s, Hs, leaf, c4);
}

// ---------------------------------------------------------------------------
// The 3D step with shared line reconstructions (launch option value 2): the
// workgroup, flux store and cell finishing of k_step3d_wg, with face fluxes
// from tasks that reconstruct each (cell, line) once per face orientation
// and use both ends of its parabola.
//  - Plane task (z): lane (x, y) holds cell (x, y, z) and evaluates its low
//    x-face and its low y-face.  A face point takes an end of a line of the
//    cell below along the face normal (the lane before: a DPP shift of one
//    lane for x, a shuffle of 8 lanes for y) as its left state and an end of
//    a line of its own cell as its right state.  The 12 lines with an x or y
//    component serve both orientations: each is reconstructed once (18 for
//    the two orientations apart).  Lanes at x = 0 (y = 0) have no x-face
//    (y-face) of theirs; faces 0 and 8 come from the boundary tasks.
//  - Boundary task: face 0 or face 8 along x or y for the whole leaf, one
//    face per lane, evaluated as in k_step3d_wg (both sides' line ends).
//  - Column task: lane (x, y) walks up its column, carrying the right ends
//    of the 9 lines a x + b y + z of the cell below; face c - 1/2 takes the
//    carried end of e(a, b) and the left end of e(-a, -b) of cell c at point
//    (a, b).  Two tasks split the column: faces 0..3 and 4..8.
// The column task walks its lines in the direction of the face normal, not
// always in the canonical direction of the point, and parabola() gives the
// same ends either way.  The points are taken in pairs (a, b) and (-a, -b),
// whose two lines give both points' states, or in the plane task by line
// group, in the order of the Simpson sums, so each face's flux is the
// sequence of operations face_flux_3d performs: the same bits.  Each group's
// results are kept in program order (keep_order): without that a
// single-orientation plane task at 11 binary64 fields spilled 248 VGPRs,
// with it it took 300 and spilled none.
// ---------------------------------------------------------------------------

// The flux store of k_step3d_ws: k_step3d_wg's 27 planes and a spare one
// that takes the stores of lanes without a face, so that every store is
// unconditional (a conditional one lets the compiler sink the flux
// arithmetic behind it, away from the lane moves it depends on, which then
// hold their registers to the end of the task).
constexpr int WS_PLANES = FACE_PLANES + 1;
constexpr int WS_SPARE = FACE_PLANES;
template <typename T, int NF>
constexpr size_t ws3d_lds_bytes() {
  return (size_t)WS_PLANES * 64 * NF * sizeof(T);
}

// Point pairs (a, b), (-a, -b) in the order of the Simpson sums; the last is
// the centre point, a line of its own.
constexpr int WS_PA[5] = {1, 1, 0, 1, 0};
constexpr int WS_PB[5] = {1, -1, 1, 0, 0};

// Running Simpson sums of one field over the pairs: pair 0 gives
// (h(-1,-1) + h(1,1)), pair 1 adds (h(1,-1) + h(-1,1)) for the corners,
// pairs 2 and 3 do the same for the edges, the centre closes the sum.
template <typename T>
__device__ __forceinline__ void simpson_pair(int p, T hp, T hm, T& sa, T& sb, T& out) {
  if (p == 0) sa = hm + hp;
  else if (p == 1) sa = sa + (hp + hm);
  else if (p == 2) sb = hm + hp;
  else if (p == 3) sb = sb + (hm + hp);
  else out = ((sa + T(4) * sb) + T(16) * hp) / T(36);
}

// Value of the previous cell along D within the lane's cell plane, lane
// (x, y) = x + 8 y: for x, lane - 1 by a DPP row shift (the lanes without a
// source keep the value itself, so no register has to be cleared for them);
// for y, lane - 8 by a shuffle.  Lanes at the plane's first cell along D
// receive a value they never use.  (Lanes ordered (y, x), which would let y
// use the DPP shift too, measured no faster.)
__device__ __forceinline__ int row_shr1(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false);  // row_shr:1
}
template <int D, typename T>
__device__ __forceinline__ T prev_cell(T v) {
  if constexpr (D == 0) {
    if constexpr (sizeof(T) == 8) {
      const unsigned long long b = (unsigned long long)__double_as_longlong(v);
      const int lo = row_shr1((int)(unsigned)b), hi = row_shr1((int)(unsigned)(b >> 32));
      return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                              (unsigned long long)(unsigned)lo));
    } else {
      return __int_as_float(row_shr1(__float_as_int(v)));
    }
  } else {
    return __shfl_up(v, 8, 64);
  }
}

// Kurganov-Tadmor flux of one passive field at a point from the point's
// velocities and half signal speed.
template <typename T>
__device__ __forceinline__ T passive_flux(T ul, T ur, T vl, T vr, T ha) {
  return T(0.5) * (ul * vl + ur * vr) - ha * (ur - ul);
}

// Plane task: faces 1..7 along x and along y of cell plane z into Hs, lane
// (x, y) holding cell (x, y, z), with the lines that serve both orientations
// reconstructed once:
//   body diagonals L0 (1,1,1), L1 (1,-1,-1), L2 (1,1,-1), L3 (1,-1,1): the
//     corner points of the x-faces and of the y-faces;
//   M0 (1,0,1), M1 (1,0,-1): the x-faces' edge points (0, +-1);
//   N0 (0,1,1), N1 (0,1,-1): the y-faces' edge points (0, +-1);
//   P0 (1,1,0), P1 (1,-1,0): the edge points (+-1, 0) of both;
//   (1,0,0) and (0,1,0): the centres.
// 12 reconstructions per cell for the two orientations instead of 18.  A
// point's left state is an end of the cell below along the face normal (x:
// a DPP shift of one lane, y: a shuffle of 8 lanes), its right state an end
// of its own cell; which end follows from the line's canonical direction.
template <typename T>
struct XYAcc {
  T xc, yc, xe, ye;  // corner and edge sums of the x- and y-face
};

template <typename T, int NF>
__device__ __forceinline__ void ws_plane_xy(const Phys<T>& ph, const T* __restrict__ Gt,
                                            size_t fsG, int z, int lane,
                                            T (&Hs)[WS_PLANES][NF][64], bool& bad) {
  constexpr int SX = 1, SY = TW, SZ = TW * TW;
  const int x = lane & 7, y = lane >> 3;
  const int t = tile_at(x, y, z);
  XYAcc<T> acc[NF];
  T Hx[NF], Hy[NF];
  bool bx = false, by = false;
  // ---- body diagonals: corners of both orientations
  {
    constexpr int s0 = SX + SY + SZ, s1 = SX - SY - SZ, s2 = SX + SY - SZ, s3 = SX - SY + SZ;
    T vl[8], vr[8], ha[8];  // points: x (1,1) (-1,-1) (1,-1) (-1,1), y the same
    {
      T xL[4][NF_CORE], xR[4][NF_CORE], yL[4][NF_CORE], yR[4][NF_CORE];
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        T l0, h0, l1, h1, l2, h2, l3, h3;
        const T* q = Gt + f * fsG + t;
        parabola(q, s0, l0, h0);
        parabola(q, s1, l1, h1);
        parabola(q, s2, l2, h2);
        parabola(q, s3, l3, h3);
        xL[0][f] = prev_cell<0>(h0); xR[0][f] = l1;  // x (1,1)
        xL[1][f] = prev_cell<0>(h1); xR[1][f] = l0;  // x (-1,-1)
        xL[2][f] = prev_cell<0>(h2); xR[2][f] = l3;  // x (1,-1)
        xL[3][f] = prev_cell<0>(h3); xR[3][f] = l2;  // x (-1,1)
        yL[0][f] = prev_cell<1>(h0); yR[0][f] = h3;  // y (1,1)
        yL[1][f] = prev_cell<1>(l3); yR[1][f] = l0;  // y (-1,-1)
        yL[2][f] = prev_cell<1>(h2); yR[2][f] = h1;  // y (1,-1)
        yL[3][f] = prev_cell<1>(l1); yR[3][f] = l2;  // y (-1,1)
      }
      T hx[4][NF_CORE], hy[4][NF_CORE];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        core_flux(ph, 0, xL[q], xR[q], hx[q], vl[q], vr[q], ha[q], bx);
        core_flux(ph, 1, yL[q], yR[q], hy[q], vl[4 + q], vr[4 + q], ha[4 + q], by);
      }
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        acc[f].xc = (hx[1][f] + hx[0][f]) + (hx[2][f] + hx[3][f]);
        acc[f].yc = (hy[1][f] + hy[0][f]) + (hy[2][f] + hy[3][f]);
        keep_order(acc[f].xc);
        keep_order(acc[f].yc);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        keep_order(vl[q]);
        keep_order(vr[q]);
        keep_order(ha[q]);
      }
    }
#pragma unroll
    for (int f = NF_CORE; f < NF; ++f) {
      T l0, h0, l1, h1, l2, h2, l3, h3;
      const T* q = Gt + f * fsG + t;
      parabola(q, s0, l0, h0);
      parabola(q, s1, l1, h1);
      parabola(q, s2, l2, h2);
      parabola(q, s3, l3, h3);
      const T x0 = passive_flux(prev_cell<0>(h0), l1, vl[0], vr[0], ha[0]);
      const T x1 = passive_flux(prev_cell<0>(h1), l0, vl[1], vr[1], ha[1]);
      const T x2 = passive_flux(prev_cell<0>(h2), l3, vl[2], vr[2], ha[2]);
      const T x3 = passive_flux(prev_cell<0>(h3), l2, vl[3], vr[3], ha[3]);
      const T y0 = passive_flux(prev_cell<1>(h0), h3, vl[4], vr[4], ha[4]);
      const T y1 = passive_flux(prev_cell<1>(l3), l0, vl[5], vr[5], ha[5]);
      const T y2 = passive_flux(prev_cell<1>(h2), h1, vl[6], vr[6], ha[6]);
      const T y3 = passive_flux(prev_cell<1>(l1), l2, vl[7], vr[7], ha[7]);
      acc[f].xc = (x1 + x0) + (x2 + x3);
      acc[f].yc = (y1 + y0) + (y2 + y3);
      keep_order(acc[f].xc);
      keep_order(acc[f].yc);
    }
  }
  // ---- two-line groups: edges.  G = 0: M (x-faces' (0, +-1)), G = 1: N
  // (y-faces' (0, +-1)), G = 2: P ((+-1, 0) of both)
#pragma unroll
  for (int G = 0; G < 3; ++G) {
    const int sA = G == 0 ? SX + SZ : (G == 1 ? SY + SZ : SX + SY);
    const int sB = G == 0 ? SX - SZ : (G == 1 ? SY - SZ : SX - SY);
    // points per group: M: x (0,-1) [L hi(M1)@x-1, R lo(M0)], x (0,1) [L hi(M0)@x-1, R lo(M1)]
    //                   N: y (0,-1) [L hi(N1)@y-1, R lo(N0)], y (0,1) [L hi(N0)@y-1, R lo(N1)]
    //                   P: x (-1,0) [L hi(P1)@x-1, R lo(P0)], x (1,0) [L hi(P0)@x-1, R lo(P1)],
    //                      y (-1,0) [L lo(P1)@y-1, R lo(P0)], y (1,0) [L hi(P0)@y-1, R hi(P1)]
    constexpr int NP = 4;
    T vl[NP], vr[NP], ha[NP];
    {
      T L[NP][NF_CORE], R[NP][NF_CORE];
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        T lA, hA, lB, hB;
        const T* q = Gt + f * fsG + t;
        parabola(q, sA, lA, hA);
        parabola(q, sB, lB, hB);
        if (G == 0) {
          L[0][f] = prev_cell<0>(hB); R[0][f] = lA;
          L[1][f] = prev_cell<0>(hA); R[1][f] = lB;
        } else if (G == 1) {
          L[0][f] = prev_cell<1>(hB); R[0][f] = lA;
          L[1][f] = prev_cell<1>(hA); R[1][f] = lB;
        } else {
          L[0][f] = prev_cell<0>(hB); R[0][f] = lA;
          L[1][f] = prev_cell<0>(hA); R[1][f] = lB;
          L[2][f] = prev_cell<1>(lB); R[2][f] = lA;
          L[3][f] = prev_cell<1>(hA); R[3][f] = hB;
        }
      }
      T h[NP][NF_CORE];
#pragma unroll
      for (int q = 0; q < (G == 2 ? 4 : 2); ++q) {
        const int D = G == 0 ? 0 : (G == 1 ? 1 : (q < 2 ? 0 : 1));
        core_flux(ph, D, L[q], R[q], h[q], vl[q], vr[q], ha[q], D == 0 ? bx : by);
      }
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        if (G == 0) acc[f].xe = h[0][f] + h[1][f];
        else if (G == 1) acc[f].ye = h[0][f] + h[1][f];
        else {
          acc[f].xe = acc[f].xe + (h[0][f] + h[1][f]);
          acc[f].ye = acc[f].ye + (h[2][f] + h[3][f]);
        }
        keep_order(acc[f].xe);
        keep_order(acc[f].ye);
      }
#pragma unroll
      for (int q = 0; q < (G == 2 ? 4 : 2); ++q) {
        keep_order(vl[q]);
        keep_order(vr[q]);
        keep_order(ha[q]);
      }
    }
#pragma unroll
    for (int f = NF_CORE; f < NF; ++f) {
      T lA, hA, lB, hB;
      const T* q = Gt + f * fsG + t;
      parabola(q, sA, lA, hA);
      parabola(q, sB, lB, hB);
      if (G == 0) {
        acc[f].xe = passive_flux(prev_cell<0>(hB), lA, vl[0], vr[0], ha[0]) +
                    passive_flux(prev_cell<0>(hA), lB, vl[1], vr[1], ha[1]);
      } else if (G == 1) {
        acc[f].ye = passive_flux(prev_cell<1>(hB), lA, vl[0], vr[0], ha[0]) +
                    passive_flux(prev_cell<1>(hA), lB, vl[1], vr[1], ha[1]);
      } else {
        acc[f].xe = acc[f].xe + (passive_flux(prev_cell<0>(hB), lA, vl[0], vr[0], ha[0]) +
                                 passive_flux(prev_cell<0>(hA), lB, vl[1], vr[1], ha[1]));
        acc[f].ye = acc[f].ye + (passive_flux(prev_cell<1>(lB), lA, vl[2], vr[2], ha[2]) +
                                 passive_flux(prev_cell<1>(hA), hB, vl[3], vr[3], ha[3]));
      }
      keep_order(acc[f].xe);
      keep_order(acc[f].ye);
    }
  }
  // ---- centres: (1,0,0) for x, (0,1,0) for y
  {
    T vlx, vrx, hax, vly, vry, hay;
    {
      T XL[NF_CORE], XR[NF_CORE], YL[NF_CORE], YR[NF_CORE], hx[NF_CORE], hy[NF_CORE];
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        T lx, hxe, ly, hye;
        const T* q = Gt + f * fsG + t;
        parabola(q, SX, lx, hxe);
        parabola(q, SY, ly, hye);
        XL[f] = prev_cell<0>(hxe); XR[f] = lx;
        YL[f] = prev_cell<1>(hye); YR[f] = ly;
      }
      core_flux(ph, 0, XL, XR, hx, vlx, vrx, hax, bx);
      core_flux(ph, 1, YL, YR, hy, vly, vry, hay, by);
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        Hx[f] = ((acc[f].xc + T(4) * acc[f].xe) + T(16) * hx[f]) / T(36);
        Hy[f] = ((acc[f].yc + T(4) * acc[f].ye) + T(16) * hy[f]) / T(36);
        keep_order(Hx[f]);
        keep_order(Hy[f]);
      }
      keep_order(vlx); keep_order(vrx); keep_order(hax);
      keep_order(vly); keep_order(vry); keep_order(hay);
    }
#pragma unroll
    for (int f = NF_CORE; f < NF; ++f) {
      T lx, hxe, ly, hye;
      const T* q = Gt + f * fsG + t;
      parabola(q, SX, lx, hxe);
      parabola(q, SY, ly, hye);
      const T cx = passive_flux(prev_cell<0>(hxe), lx, vlx, vrx, hax);
      const T cy = passive_flux(prev_cell<1>(hye), ly, vly, vry, hay);
      Hx[f] = ((acc[f].xc + T(4) * acc[f].xe) + T(16) * cx) / T(36);
      Hy[f] = ((acc[f].yc + T(4) * acc[f].ye) + T(16) * cy) / T(36);
      keep_order(Hx[f]);
      keep_order(Hy[f]);
    }
  }
  bad |= (bx && x != 0) || (by && y != 0);
  const int sx = x != 0 ? z : WS_SPARE, sy = y != 0 ? 9 + z : WS_SPARE;
#pragma unroll
  for (int f = 0; f < NF; ++f) Hs[sx][f][lane] = Hx[f];
#pragma unroll
  for (int f = 0; f < NF; ++f) Hs[sy][f][lane] = Hy[f];
}

// Boundary task k (0: x-face 0, 1: x-face 8, 2: y-face 0, 3: y-face 8):
// lane (a, b) is the face's transverse position ((y, z) or (x, z)).
template <typename T, int NF>
__device__ __forceinline__ void ws_boundary(const GridArgs& g, const Phys<T>& ph,
                                            const T* __restrict__ Gt, size_t fsG, int leaf,
                                            int k, int lane, T (&Hs)[WS_PLANES][NF][64],
                                            bool& bad) {
  const int a = lane & 7, b = lane >> 3;
  const bool hi = (k & 1) != 0;
  T H[NF];
  if (k < 2) {
    face_flux_3d<T, NF, 0>(ph, Gt, fsG, hi ? tile_at(SUB - 1, a, b) : tile_at(-1, a, b), H, bad);
    if (g.reg) record_face<T, NF>(g, face_slots_3d(g, leaf, 0), hi ? SUB : 0, a, b, H);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (hi) Hs[SUB][f][lane] = H[f];
      else Hs[b][f][8 * a] = H[f];  // face 0 of row (y, z) = (a, b)
    }
  } else {
    face_flux_3d<T, NF, 1>(ph, Gt, fsG, hi ? tile_at(a, SUB - 1, b) : tile_at(a, -1, b), H, bad);
    if (g.reg) record_face<T, NF>(g, face_slots_3d(g, leaf, 1), hi ? SUB : 0, a, b, H);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (hi) Hs[9 + SUB][f][lane] = H[f];
      else Hs[9 + b][f][a] = H[f];  // face 0 of column (x, z) = (a, b)
    }
  }
}

// Column task: z-faces c0..c1 of lane (x, y)'s column into Hs, in the
// field order of the plane task.  The cell below face c0 only fills the
// carry.
template <typename T, int NF>
__device__ __forceinline__ void ws_column(const GridArgs& g, const Phys<T>& ph,
                                          const T* __restrict__ Gt, size_t fsG, int leaf, int c0,
                                          int c1, int lane, T (&Hs)[WS_PLANES][NF][64],
                                          bool& bad) {
  constexpr int SU = 1, SV = TW, SD = TW * TW;
  const int x = lane & 7, y = lane >> 3;
  // right ends of the cell below: [2p] line e(a, b), [2p + 1] line e(-a, -b)
  T cr[9][NF];
  {
    const int t = tile_at(x, y, c0 - 1);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
      for (int p = 0; p < 5; ++p) {
        T l;
        parabola(Gt + f * fsG + t, SD + WS_PA[p] * SU + WS_PB[p] * SV, l, cr[2 * p][f]);
        keep_order(cr[2 * p][f]);
        if (p < 4) {
          parabola(Gt + f * fsG + t, SD - WS_PA[p] * SU - WS_PB[p] * SV, l, cr[2 * p + 1][f]);
          keep_order(cr[2 * p + 1][f]);
        }
      }
    }
  }
#pragma unroll 1
  for (int c = c0; c <= c1; ++c) {
    const int t = tile_at(x, y, c);
    T sa[NF_CORE], sb[NF_CORE], H[NF];
    T vl[9], vr[9], ha[9];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const int sA = SD + WS_PA[p] * SU + WS_PB[p] * SV;
      const int sB = SD - WS_PA[p] * SU - WS_PB[p] * SV;
      T ULp[NF_CORE], URp[NF_CORE], ULm[NF_CORE], URm[NF_CORE];
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        T lA, rA;
        parabola(Gt + f * fsG + t, sA, lA, rA);
        ULp[f] = cr[2 * p][f];
        cr[2 * p][f] = rA;
        if (p < 4) {
          T lB, rB;
          parabola(Gt + f * fsG + t, sB, lB, rB);
          URp[f] = lB;
          ULm[f] = cr[2 * p + 1][f];
          cr[2 * p + 1][f] = rB;
          URm[f] = lA;
        } else {
          URp[f] = lA;
        }
      }
      T Hp[NF_CORE], Hm[NF_CORE];
      core_flux(ph, 2, ULp, URp, Hp, vl[2 * p], vr[2 * p], ha[2 * p], bad);
      if (p < 4)
        core_flux(ph, 2, ULm, URm, Hm, vl[2 * p + 1], vr[2 * p + 1], ha[2 * p + 1], bad);
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        simpson_pair(p, Hp[f], p < 4 ? Hm[f] : T(0), sa[f], sb[f], H[f]);
        keep_order(p < 2 ? sa[f] : (p < 4 ? sb[f] : H[f]));
      }
      keep_order(vl[2 * p]);
      keep_order(vr[2 * p]);
      keep_order(ha[2 * p]);
      if (p < 4) {
        keep_order(vl[2 * p + 1]);
        keep_order(vr[2 * p + 1]);
        keep_order(ha[2 * p + 1]);
      }
#pragma unroll
      for (int f = 0; f < NF_CORE; ++f) {
        keep_order(cr[2 * p][f]);
        if (p < 4) keep_order(cr[2 * p + 1][f]);
      }
    }
#pragma unroll
    for (int f = NF_CORE; f < NF; ++f) {
      T fa = T(0), fb = T(0);
#pragma unroll
      for (int p = 0; p < 5; ++p) {
        const int sA = SD + WS_PA[p] * SU + WS_PB[p] * SV;
        const int sB = SD - WS_PA[p] * SU - WS_PB[p] * SV;
        T lA, rA, hp, hm = T(0);
        parabola(Gt + f * fsG + t, sA, lA, rA);
        const T ulp = cr[2 * p][f];
        cr[2 * p][f] = rA;
        if (p < 4) {
          T lB, rB;
          parabola(Gt + f * fsG + t, sB, lB, rB);
          const T ulm = cr[2 * p + 1][f];
          cr[2 * p + 1][f] = rB;
          hp = passive_flux(ulp, lB, vl[2 * p], vr[2 * p], ha[2 * p]);
          hm = passive_flux(ulm, lA, vl[2 * p + 1], vr[2 * p + 1], ha[2 * p + 1]);
        } else {
          hp = passive_flux(ulp, lA, vl[2 * p], vr[2 * p], ha[2 * p]);
        }
        simpson_pair(p, hp, hm, fa, fb, H[f]);
        keep_order(p < 2 ? fa : (p < 4 ? fb : H[f]));
        keep_order(cr[2 * p][f]);
        if (p < 4) keep_order(cr[2 * p + 1][f]);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) Hs[18 + c][f][lane] = H[f];
    if (g.reg && (c == 0 || c == SUB))
      record_face<T, NF>(g, face_slots_3d(g, leaf, 2), c, x, y, H);
  }
}

// Work of each wavefront, in this order (the boundary faces, which span the
// whole tile, come last; by VALU instructions at 11 binary64 fields the
// lists are 68 k, 58 k, 69 k and 70 k, and no other split of these tasks
// does better):
//   0: z-faces 4..8, y-face 8
//   1: z-faces 0..3, plane 7
//   2: planes 0..3, x-face 8
//   3: planes 4..6, x-face 0, y-face 0
// written out per wavefront, not as a list of tasks in one loop: in a loop
// the compiler keeps every task's loop-invariant values in registers
// through all of them.
// binary32 at two workgroups per CU where two flux stores fit in LDS (256
// registers; the store is 77 KB at 11 fields), binary64 at one.
template <typename T, int NF>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 && 2 * ws3d_lds_bytes<T, NF>() <= 160 * 1024)
                                           ? 2 : 1)
    k_step3d_ws(StepArgs s, const T* __restrict__ G) {
  __shared__ T Hs[WS_PLANES][NF][64];  // the layout of k_step3d_wg and a spare plane
  const GridArgs& g = s.g;
  const int leaf = s.leaf_base + blockIdx.x;
  if (leaf >= g.n_leaves) return;  // uniform over the workgroup
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  Phys<T> ph;
  ph.gamma = (T)g.gamma;
  ph.gm1 = (T)(g.gamma - 1.0);
  ph.eta1 = (T)g.eta1;
  const size_t fsG = (size_t)g.n_leaves * TILE;
  const T* __restrict__ Gt = G + (size_t)leaf * TILE;
  bool bad = false;
  if (wave < 2)
    ws_column<T, NF>(g, ph, Gt, fsG, leaf, wave == 0 ? 4 : 0, wave == 0 ? SUB : 3, lane, Hs, bad);
  const int z0 = wave == 1 ? 7 : (wave == 2 ? 0 : 4);
  const int z1 = wave == 0 ? -1 : (wave == 1 ? 7 : (wave == 2 ? 3 : 6));
#pragma unroll 1
  for (int z = z0; z <= z1; ++z) ws_plane_xy<T, NF>(ph, Gt, fsG, z, lane, Hs, bad);
  // boundary tasks k0, k0 + 2, ... up to k1
  const int k0 = wave == 0 ? 3 : (wave == 3 ? 0 : 1);
  const int k1 = wave == 0 ? 3 : (wave == 1 ? 0 : (wave == 2 ? 1 : 2));
#pragma unroll 1
  for (int k = k0; k <= k1; k += 2) ws_boundary<T, NF>(g, ph, Gt, fsG, leaf, k, lane, Hs, bad);
  if (g.status && __any(bad) && lane == 0) atomicOr(g.status, (int)HYDRO_STATUS_UNPHYSICAL);
  __syncthreads();
  finish_leaf_3d<T, NF, WS_PLANES>(s, Hs, leaf, c4);
}

// Launch of the 3D step: where the workgroup forms' flux store fits in LDS
// (binary64 up to 11 fields, binary32 up to 16), the form wg asks for (1:
// k_step3d_wg, 2: k_step3d_ws); else, or for wg == 0, k_step3d.
template <typename T, int NF>
hipError_t launch_step3d_one(const StepArgs& a, int blocks, const T* G, int wg, hipStream_t st) {
  if constexpr (wg3d_lds_bytes<T, NF>() <= 160 * 1024) {
    if (wg == 1) {
      hipLaunchKernelGGL((k_step3d_wg<T, NF>), dim3(blocks), dim3(256), 0, st, a, G);
      return hipGetLastError();
    }
  }
  if constexpr (ws3d_lds_bytes<T, NF>() <= 160 * 1024) {
    if (wg == 2) {
      hipLaunchKernelGGL((k_step3d_ws<T, NF>), dim3(blocks), dim3(256), 0, st, a, G);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_step3d<T, NF>), dim3(blocks), dim3(64), 0, st, a, G);
  return hipGetLastError();
}

#define OCTOHYDRO_3D_EXTERN(T, n) \
  extern template hipError_t launch_step3d_one<T, n>(const StepArgs&, int, const T*, int, \
                                                     hipStream_t);
#define OCTOHYDRO_3D_EXTERN_ALL(T)                                                    \
  OCTOHYDRO_3D_EXTERN(T, 6) OCTOHYDRO_3D_EXTERN(T, 7) OCTOHYDRO_3D_EXTERN(T, 8)       \
  OCTOHYDRO_3D_EXTERN(T, 9) OCTOHYDRO_3D_EXTERN(T, 10) OCTOHYDRO_3D_EXTERN(T, 11)     \
  OCTOHYDRO_3D_EXTERN(T, 12) OCTOHYDRO_3D_EXTERN(T, 13) OCTOHYDRO_3D_EXTERN(T, 14)    \
  OCTOHYDRO_3D_EXTERN(T, 15) OCTOHYDRO_3D_EXTERN(T, 16)
OCTOHYDRO_3D_EXTERN_ALL(double)
OCTOHYDRO_3D_EXTERN_ALL(float)
#undef OCTOHYDRO_3D_EXTERN_ALL
#undef OCTOHYDRO_3D_EXTERN

template <typename T>
inline hipError_t launch_step3d_t(const StepArgs& a, int blocks, const T* G, int wg,
                                  hipStream_t st) {
  switch (a.g.nf) {
#define OCTOHYDRO_CASE3D(n) \
  case n: return launch_step3d_one<T, n>(a, blocks, G, wg, st);
    OCTOHYDRO_CASE3D(6) OCTOHYDRO_CASE3D(7) OCTOHYDRO_CASE3D(8) OCTOHYDRO_CASE3D(9)
    OCTOHYDRO_CASE3D(10) OCTOHYDRO_CASE3D(11) OCTOHYDRO_CASE3D(12) OCTOHYDRO_CASE3D(13)
    OCTOHYDRO_CASE3D(14) OCTOHYDRO_CASE3D(15) OCTOHYDRO_CASE3D(16)
#undef OCTOHYDRO_CASE3D
    default: return hipErrorInvalidValue;
  }
}

}  // namespace octohydro
