// liboctohydro: octree hydro step for gfx950 (AMD Instinct MI355X).  This
// unit holds the C-ABI entry points, the host-side launch logic and the
// small kernels; the method's device code and the step kernels are in
// octohydro_kernels.h (the 3D step's in octohydro_kernels3d.h), instantiated
// in the k_step_*.hip and k_step3d*.hip units.
//
// Kernels behind the C-ABI in include/octohydro.h:
//   k_fill     ghost fill into materialised 14^3 tiles (hydro_fill_ghosts)
//   k_restrict restricted copies of the refined nodes, before a substep
//              (within an RK3 step the substeps leave them after the first)
//   k_step     fused substep: neighbour gather + PPM + Kurganov-Tadmor flux +
//              flux divergence + Runge-Kutta stage combination (hydro_step)
//   k_step3d   the same with the full 3D reconstruction and face quadrature
//   k_reflux   coarse-fine flux correction
//   k_cfl      global time step: per-cell dx / signal speed, wave64 min, one
//              64-bit atomic min per workgroup (hydro_cfl_dt)
//   k_totals   conserved totals with double-double accumulation
//
// The method (paper Sec. IV-C, V-B-1, VI; textbook forms named in the public
// header) is evaluated operation by operation in the order the method states:
// in binary64 every operation is one IEEE-754 operation rounded once, with no
// FMA contraction, so the binary64 path reproduces a plain sequential
// evaluation bit for bit.
//
// Layout in HBM: structure of arrays, field-major: U[f][leaf][z][y][x].
// One 64-lane wavefront owns one leaf in k_step, in two z-halves: lanes
// stream the x- and y-pencils of the half's planes, then the z-pencils, each
// lane its 14 values (3 ghosts, 8 interior, 3 ghosts) through the PPM
// recurrences in registers; ghost values are read straight from the
// neighbour leaf in global memory (face neighbours only: dimension-by-
// dimension reconstruction never needs edge or corner ghosts).  The flux
// differences meet in an LDS accumulator, and the z-pencils finish the
// update and write Uout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "octohydro.h"
#include "octohydro_internal.h"
#include "octohydro_kernels.h"

namespace octohydro {

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

// Time step of a chained RK3 step: dt[0] = cfl * dt[1], the CFL minimum of
// the step's input left by the previous step; dt[1] = +inf, ready for the
// minimum of the step's output.
__global__ void k_dt_take(double* dt, double cfl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dt[0] = cfl * dt[1];
    *reinterpret_cast<unsigned long long*>(dt + 1) = 0x7FF0000000000000ull;
  }
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
      // the children the 3-layer halo in this direction reads must exist:
      // along an axis with offset +1 the low child, -1 the high child, 0
      // both (the ghost fill and the restriction read them unchecked)
      const int slot = (int)(i % 27);
      const int r[3] = {slot % 3 - 1, (slot / 3) % 3 - 1, slot / 9 - 1};
      if (ok)
        for (int c = 0; c < 8; ++c) {
          const int ch = g.children[8 * id + c];
          bool needed = true;
          for (int k = 0; k < 3; ++k) {
            const int bit = (c >> k) & 1;
            needed = needed && (r[k] == 0 || bit == (r[k] > 0 ? 0 : 1));
          }
          ok = ok && ch >= -1 && ch < g.n_leaves && (!needed || ch >= 0);
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
  g.leaf_node = gr->leaf_node_dev;
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

// Ghost fill (hydro_fill_ghosts) into materialised tiles.
// One workgroup of FILL_THREADS per leaf: 512 keeps as many wavefronts in
// flight per CU as 256 with half as many leaves, so more of the neighbour
// cells a tile reads are still in L2 (binary64 6.29 -> 6.04 ms on the
// 65,535-leaf case, binary32 unchanged; 1024: 6.35 and 4.37 ms).
constexpr int FILL_THREADS = 512;
// Each thread takes tile cells t, t + FILL_THREADS, ..., works
// out where the cell's value comes from once (the leaf itself, a same-level
// or coarser leaf, or the 8 cells of a refined neighbour's child) and copies
// or restricts that source in every field.  Consecutive threads hold
// consecutive tile cells, so a wavefront's writes and most of its reads are
// contiguous rows.  The tile stores are non-temporal: nothing in this kernel
// reads a tile again, and streaming the tiles past L2 leaves it to the
// neighbour cells that other tiles read (65,535-leaf case: 7.85 -> 6.29 ms
// in binary64, 4.85 -> 3.93 ms in binary32, fetched bytes 20.6 -> 16.0 GB;
// fewer workgroups per CU, for a smaller working set, measured slower).
template <typename T>
__global__ void __launch_bounds__(FILL_THREADS) k_fill(GridArgs g, const T* __restrict__ U,
                                              T* __restrict__ G, int remap) {
  const int leaf = leaf_of_block(blockIdx.x, g.n_leaves, remap);
  const int4 c4 = reinterpret_cast<const int4*>(g.coord)[leaf];
  const int ic[3] = {c4.y, c4.z, c4.w};
  const int blocks = g.base << c4.x;
  const size_t fsU = (size_t)g.n_leaves * CELLS, fsG = (size_t)g.n_leaves * TILE;
  T* __restrict__ Gl = G + (size_t)leaf * TILE;
  for (int t = threadIdx.x; t < TILE; t += blockDim.x) {
    const int tp[3] = {t % TW, (t / TW) % TW, t / (TW * TW)};
    int r[3], l[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r[k] = tp[k] < GH ? -1 : (tp[k] >= GH + SUB ? 1 : 0);
      l[k] = tp[k] - GH - SUB * r[k];
    }
    const int slot = (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
    const int kind = slot == 13 ? (int)HYDRO_SAME_LEAF : (int)g.kind[27 * leaf + slot];
    const int id = slot == 13 ? leaf : g.nbr[27 * leaf + slot];
    if (kind == HYDRO_SAME_REFINED) {
      for (int f = 0; f < g.nf; ++f)
        __builtin_nontemporal_store(
            neighbour_value<T>(g, U + f * fsU, leaf, ic, blocks, kind, id, r, l), &Gl[f * fsG + t]);
    } else {
      // a copy: the cell itself, a same-level cell or the covering coarse
      // cell; every field's load is issued before the first store
      const T* __restrict__ src = U;
      size_t o;
      if (kind == HYDRO_SAME_LEAF) {
        o = (size_t)id * CELLS + l[2] * 64 + l[1] * 8 + l[0];
      } else {
        int c[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int nb = wrap(ic[k] + r[k], blocks);
          c[k] = 4 * (nb & 1) + (l[k] >> 1);
        }
        o = (size_t)id * CELLS + c[2] * 64 + c[1] * 8 + c[0];
      }
      T v[16];
#pragma unroll
      for (int f = 0; f < 16; ++f)
        if (f < g.nf) v[f] = src[f * fsU + o];
#pragma unroll
      for (int f = 0; f < 16; ++f)
        if (f < g.nf) __builtin_nontemporal_store(v[f], &Gl[f * fsG + t]);
    }
  }
}

// Ghosted 14^3 tiles of U into G (all 26 ghost regions).
// Leaves go to the XCDs in contiguous Morton ranges (remap mode 1), so that a
// tile's neighbour cells are mostly read on the XCD that reads them for the
// neighbour's own tile: 8.12 -> 7.85 ms per binary64 fill of the 65535-leaf
// case (binary32 unchanged).
constexpr int FILL_REMAP = 1;
static int fill_launch(const hydro_grid* gr, const void* U, void* G, hipStream_t st) {
  const GridArgs g = grid_args(gr);
  if (gr->dtype == HYDRO_F64)
    hipLaunchKernelGGL(k_fill<double>, dim3(g.n_leaves), dim3(FILL_THREADS), 0, st, g,
                       static_cast<const double*>(U), static_cast<double*>(G), FILL_REMAP);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(g.n_leaves), dim3(FILL_THREADS), 0, st, g,
                       static_cast<const float*>(U), static_cast<float*>(G), FILL_REMAP);
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
  int waves_per_leaf = 1;
  int cfl_epilogue = 1;
  int fused_restrict = 1;
  int recon3d_wg = 2;
};
static Options g_opts[2][17];
static std::mutex g_opts_mu;

static Options get_options(int dtype, int nf) {
  std::lock_guard<std::mutex> lk(g_opts_mu);
  return g_opts[dtype][nf];
}

// Whether the step kernel itself leaves the CFL minimum of its output: the
// axis reconstruction without the flux correction (the correction changes
// cells after the kernel; the 3D step has no epilogue) when the launch
// option asks for it; else a pass of k_cfl over the output does it.
static bool cfl_in_kernel(const hydro_grid* gr, const StepArgs& a) {
  return gr->reconstruction == HYDRO_RECON_AXIS && a.g.reg == nullptr &&
         get_options(gr->dtype, gr->n_fields).cfl_epilogue != 0;
}

static hipError_t launch_step(StepArgs a, int dtype, int blocks, hipStream_t st) {
  const Options o = get_options(dtype, a.g.nf);
  if (a.remap) a.remap = o.xcd_remap;
  const StepShape sh{o.waves_per_simd, o.waves_per_leaf};
  if (a.dt_next && a.node_out) return hipErrorInvalidValue;  // no kernel does both
  if (a.dt_next)
    return dtype == HYDRO_F64 ? launch_step_f64_cfl(a, blocks, sh, st)
                              : launch_step_f32_cfl(a, blocks, sh, st);
  if (a.node_out)
    return dtype == HYDRO_F64 ? launch_step_f64_restrict(a, blocks, sh, st)
                              : launch_step_f32_restrict(a, blocks, sh, st);
  return dtype == HYDRO_F64 ? launch_step_f64(a, blocks, sh, st)
                            : launch_step_f32(a, blocks, sh, st);
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
  if (flags & ~(HYDRO_FLAG_VALIDATE | HYDRO_FLAG_NODES_READY | HYDRO_FLAG_CFL_NEXT))
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
    if (gr->node_state2_dev && (gr->node_state2_dev == gr->node_state_dev ||
                                gr->node_state2_dev == Uk || gr->node_state2_dev == Uout ||
                                (U0 && gr->node_state2_dev == U0)))
      return fail(HYDRO_E_ARG, "%s: node_state2_dev aliases another buffer", fn);
  }
  a.g = grid_args(gr);
  a.U0 = U0;
  a.Uk = Uk;
  a.Uout = Uout;
  a.dt = dt;
  a.beta = beta;
  a.leaf_base = 0;
  a.remap = 1;
  a.dt_next = nullptr;
  a.node_out = nullptr;
  return HYDRO_OK;
}

// *dt = cfl * (CFL minimum of U); with cfl == 0 the raw minimum is left.
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
  if (cfl != 0.0) {
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(64), 0, st, dt, cfl);
    HIP_TRY(hipGetLastError());
  }
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
    HIP_TRY(launch_step3d(a, gr->dtype, blocks, gr->ghost_tile_dev,
                          get_options(gr->dtype, gr->n_fields).recon3d_wg, st));
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
  const bool chained = gr->cfl_epilogue != 0;
  if (chained) {
    // dt[0] from the minimum of Un that the previous step left in dt[1]
    if (cfl > 0.0)
      hipLaunchKernelGGL(k_dt_take, dim3(1), dim3(64), 0, st, dt, cfl);
    else
      hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, st, dt + 1);
    HIP_TRY(hipGetLastError());
  } else if (cfl > 0.0) {
    rc = cfl_launch(gr, Un, cfl, dt, st);
    if (rc) return rc;
  }
  // restricted node copies: made by a pass before each substep, or, with a
  // second node buffer, only before the first, the first two substeps then
  // leaving those of their outputs for the next (not with the flux
  // correction, which changes cells after the kernel)
  const bool fused = gr->node_state2_dev && gr->leaf_node_dev && gr->n_nodes > 0 &&
                     gr->reconstruction == HYDRO_RECON_AXIS && !a.g.reg &&
                     get_options(gr->dtype, gr->n_fields).fused_restrict != 0;
  if (fused) a.node_out = gr->node_state2_dev;
  if ((rc = substep_kernels(gr, a, gr->n_leaves, true, st))) return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
  a.U0 = Un;
  a.Uk = W1;
  a.Uout = W2;
  a.beta = 0.25;
  if (fused) {
    a.g.rstate = gr->node_state2_dev;
    a.node_out = gr->node_state_dev;
  }
  if ((rc = substep_kernels(gr, a, gr->n_leaves, !fused, st))) return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
  a.Uk = W2;
  a.Uout = Unext;
  a.beta = 2.0 / 3.0;
  if (fused) {
    a.g.rstate = gr->node_state_dev;
    a.node_out = nullptr;
  }
  if (chained && cfl_in_kernel(gr, a)) a.dt_next = dt + 1;
  if ((rc = substep_kernels(gr, a, gr->n_leaves, !fused, st))) return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
  if (chained && !a.dt_next) return cfl_launch(gr, Unext, 0.0, dt + 1, st);
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

// Partial sums of the allocation-free totals (hydro_totals_noalloc): a fixed
// device array of the library, one copy per GPU, held until the process
// ends.  Room for TOT_BLOCKS double-double partials of up to 16 fields
// (256 KiB).  Host code never passes this name to a kernel: it stands for a
// host-side shadow, and the device address of each GPU's copy comes from
// hipGetSymbolAddress (static_scratch below).
constexpr size_t NOALLOC_DOUBLES = 2 * (size_t)TOT_BLOCKS * 16;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

struct StaticScratch {
  std::mutex mu;
  std::vector<double*> ptr;  // device address of `scratch`, per device
};
static StaticScratch g_static;

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int static_scratch(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_static.mu);
  if ((int)g_static.ptr.size() <= dev) g_static.ptr.resize(dev + 1, nullptr);
  if (!g_static.ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HYDRO_E_HIP, "hipGetSymbolAddress returned no address for the scratch");
    g_static.ptr[dev] = static_cast<double*>(p);
  }
  *out = g_static.ptr[dev];
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
      if (value < 0 || value > 4096 || (value >= 2 && (value & (value - 1))))
        return fail(HYDRO_E_ARG,
                    "hydro_set_option: remap is 0, 1 or a power of two in [2, 4096]");
      o.xcd_remap = value;
      return HYDRO_OK;
    case HYDRO_OPT_3D_WORKGROUP:
      if (value < 0 || value > 2)
        return fail(HYDRO_E_ARG, "hydro_set_option: 3D workgroup form is 0, 1 or 2");
      o.recon3d_wg = value;
      return HYDRO_OK;
    case HYDRO_OPT_FUSED_RESTRICT:
      if (value != 0 && value != 1)
        return fail(HYDRO_E_ARG, "hydro_set_option: fused restriction is 0 or 1");
      o.fused_restrict = value;
      return HYDRO_OK;
    case HYDRO_OPT_CFL_EPILOGUE:
      if (value != 0 && value != 1)
        return fail(HYDRO_E_ARG, "hydro_set_option: CFL epilogue is 0 or 1");
      o.cfl_epilogue = value;
      return HYDRO_OK;
    case HYDRO_OPT_WAVES_PER_LEAF:
      if (value != 1 && value != 2)
        return fail(HYDRO_E_ARG, "hydro_set_option: wavefronts per leaf must be 1 or 2");
      if (value == 2 && n_fields == NF_CORE)
        return fail(HYDRO_E_ARG, "hydro_set_option: 2 wavefronts per leaf need passive species");
      o.waves_per_leaf = value;
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
  else if (option == HYDRO_OPT_WAVES_PER_LEAF) *value = o.waves_per_leaf;
  else if (option == HYDRO_OPT_CFL_EPILOGUE) *value = o.cfl_epilogue;
  else if (option == HYDRO_OPT_FUSED_RESTRICT) *value = o.fused_restrict;
  else if (option == HYDRO_OPT_3D_WORKGROUP) *value = o.recon3d_wg;
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
  const bool cfl_next = (flags & HYDRO_FLAG_CFL_NEXT) != 0;
  if (cfl_next) {
    if (cfl_in_kernel(gr, a)) {
      hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, st, const_cast<double*>(dt) + 1);
      HIP_TRY(hipGetLastError());
      a.dt_next = const_cast<double*>(dt) + 1;
    }
  }
  if ((rc = substep_kernels(gr, a, gr->n_leaves, !(flags & HYDRO_FLAG_NODES_READY), st)))
    return rc;
  if ((rc = reflux_launch(gr, a, st))) return rc;
  if (cfl_next && !a.dt_next) return cfl_launch(gr, Uout, 0.0, const_cast<double*>(dt) + 1, st);
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
  if (!(cfl >= 0.0)) return fail(HYDRO_E_ARG, "hydro_cfl_dt: cfl must not be negative");
  return cfl_launch(gr, U, cfl, dt, static_cast<hipStream_t>(stream));
}

// The two passes of the totals over partial sums at `part` (2 * blocks * nf
// doubles, every one of them written by the first pass before the second
// reads it: nothing needs clearing).
static int totals_launch(const GridArgs& g, int dtype, const void* U, double* part, int blocks,
                         double* totals, hipStream_t st) {
  if (dtype == HYDRO_F64)
    hipLaunchKernelGGL(k_totals<double>, dim3(blocks), dim3(TOT_THREADS), 0, st, g,
                       static_cast<const double*>(U), part);
  else
    hipLaunchKernelGGL(k_totals<float>, dim3(blocks), dim3(TOT_THREADS), 0, st, g,
                       static_cast<const float*>(U), part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(TOT_THREADS), 0, st,
                     static_cast<const double*>(part), blocks, g.nf, totals);
  HIP_TRY(hipGetLastError());
  return HYDRO_OK;
}

int hydro_totals(const hydro_grid* gr, const void* U, double* totals, void* stream) {
  clear_error();
  int rc = check_grid(gr, "hydro_totals");
  if (rc) return rc;
  if (!U || !totals) return fail(HYDRO_E_ARG, "hydro_totals: U and totals must be set");
  GridArgs g = grid_args(gr);
  const int blocks = grid_blocks(g.n_leaves, 1, TOT_BLOCKS);
  void* part = nullptr;
  rc = scratch_get(sizeof(double) * 2 * (size_t)blocks * g.nf, &part);
  if (rc) return rc;
  return totals_launch(g, gr->dtype, U, static_cast<double*>(part), blocks, totals,
                       static_cast<hipStream_t>(stream));
}

int hydro_totals_noalloc(const hydro_grid* gr, const void* U, double* totals, void* stream) {
  clear_error();
  int rc = check_grid(gr, "hydro_totals_noalloc");
  if (rc) return rc;
  if (!U || !totals) return fail(HYDRO_E_ARG, "hydro_totals_noalloc: U and totals must be set");
  GridArgs g = grid_args(gr);
  const int blocks = grid_blocks(g.n_leaves, 1, TOT_BLOCKS);
  const size_t need = 2 * (size_t)blocks * g.nf;
  if (need > NOALLOC_DOUBLES)
    return fail(HYDRO_E_ARG, "hydro_totals_noalloc: %zu partial sums exceed the fixed %zu", need,
                NOALLOC_DOUBLES);
  double* part = nullptr;
  if ((rc = static_scratch(&part))) return rc;
  return totals_launch(g, gr->dtype, U, part, blocks, totals, static_cast<hipStream_t>(stream));
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
  // both are released and the handle freed whatever either call returns
  const hipError_t e1 = h->exec ? hipGraphExecDestroy(h->exec) : hipSuccess;
  const hipError_t e2 = h->graph ? hipGraphDestroy(h->graph) : hipSuccess;
  delete h;
  const hipError_t e = e1 != hipSuccess ? e1 : e2;
  if (e != hipSuccess) return fail(HYDRO_E_HIP, "hydro_graph_destroy: %s", hipGetErrorString(e));
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
