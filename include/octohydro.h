/*
 * octohydro.h -- C-ABI of liboctohydro.so: the hydro step of an octree of
 * 8^3 sub-grids on one AMD Instinct MI355X (gfx950).
 *
 * What the library computes is the per-sub-grid hydro substep of the paper
 * "Distributed, combined CPU and GPU profiling within HPX using APEX"
 * (arXiv 2210.06437): the domain is a properly nested octree whose nodes are
 * N^3 = 8^3 Cartesian sub-grids, each refinable into 8 children at twice the
 * resolution (Sec. IV-C); every sub-grid fills its ghost cells directly from
 * its neighbours' memory (Sec. VI); the evolved variables are reconstructed
 * with PPM and fluxes come from a finite-volume central scheme for the
 * inviscid Euler equations (Sec. IV-C; kernels "reconstruct" and "flux" in
 * Sec. V-B-1); each Runge-Kutta substep computes fluxes, takes part in the
 * global time-step size and updates the variables (Sec. V-B-1,
 * compute_fluxes); a time step is three hydro substeps (Sec. I).
 * The paper names these methods only; the library implements the textbook
 * forms: Colella-Woodward PPM per conserved field, the Kurganov-Tadmor flux at
 * face centres, Shu-Osher SSP-RK3, an ideal gas with an entropy tracer and a
 * dual-energy switch.
 *
 * Conventions shared by every entry point:
 *  - Fields, in order: rho, s_x, s_y, s_z, E, tau, then passive species
 *    rho_0.. (n_fields in [6, 16]).
 *  - State arrays are structure-of-arrays [n_fields][n_leaves][8][8][8] with x
 *    fastest, in the element type named by hydro_grid.dtype.  Ghosted tiles
 *    are [n_fields][n_leaves][14][14][14] (interior at [3,11)^3).
 *  - n_leaves is at most HYDRO_MAX_LEAVES, so that one field array of a
 *    state stays below 4 GiB (kernels address it with 32-bit byte offsets);
 *    larger grids are rejected with HYDRO_E_ARG.
 *  - The domain is the periodic unit cube; a leaf at level L with coordinates
 *    (ix,iy,iz) covers level-L cells [8 ix, 8 ix + 8) x ... of width
 *    1 / (8 base 2^L).
 *  - All pointers named *_dev are device pointers owned by the caller; they
 *    must stay valid until the work queued on `stream` has finished.
 *    `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Calls are asynchronous on `stream` unless stated.  Arguments are
 *    checked on the host before anything is queued; a failing call queues
 *    nothing and returns a negative status; hydro_last_error() then gives a
 *    message (per calling thread).  No C++ exception crosses this boundary.
 */
#ifndef OCTOHYDRO_H
#define OCTOHYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HYDRO_OK 0
#define HYDRO_E_ARG (-1)          /* bad argument, caught on the host        */
#define HYDRO_E_TABLE (-2)        /* inconsistent neighbour table             */
#define HYDRO_E_UNPHYSICAL (-3)   /* rho <= 0 or p <= 0 met at a face         */
#define HYDRO_E_HIP (-4)          /* HIP runtime error (message has details)  */
#define HYDRO_E_UNSUPPORTED (-5)  /* valid request the library does not serve */

/* element types */
#define HYDRO_F64 0  /* binary64 storage and arithmetic                       */
#define HYDRO_F32 1  /* binary32 storage and face arithmetic; flux divergence,
                        stage combination, totals and time step in binary64  */

/* neighbour kinds in the 27-slot table */
#define HYDRO_SAME_LEAF 0     /* leaf at the same level: copy                */
#define HYDRO_SAME_REFINED 1  /* refined node at the same level: mean of the
                                 8 covering cells of its children            */
#define HYDRO_COARSER_LEAF 2  /* leaf one level coarser: injection           */

/* status bits written to hydro_grid.status_dev */
#define HYDRO_STATUS_UNPHYSICAL 1u
#define HYDRO_STATUS_TABLE 2u

/* reconstruction (Sec. V-B-1)
 *  HYDRO_RECON_AXIS  PPM along each axis, Kurganov-Tadmor flux at the face
 *                    centre (the default).
 *  HYDRO_RECON_3D    full three-dimensional reconstruction: values at the 26
 *                    face, edge and corner points of each cell from the same
 *                    PPM along the 13 lines of cells through it (5 cells each;
 *                    a point p/2 comes from the line along p or -p, whichever
 *                    has its first non-zero component positive), and per face
 *                    the Kurganov-Tadmor flux at its 9 points combined by the
 *                    tensor Simpson rule ((corners + 4 edges) + 16 centre)/36
 *                    with corners = (H(-1,-1)+H(1,1)) + (H(1,-1)+H(-1,1)) and
 *                    edges = (H(0,-1)+H(0,1)) + (H(-1,0)+H(1,0)).  Needs
 *                    ghost_tile_dev. */
#define HYDRO_RECON_AXIS 0
#define HYDRO_RECON_3D 1

/* flags */
#define HYDRO_FLAG_VALIDATE 1u  /* check table ids on the device and wait    */
#define HYDRO_FLAG_NODES_READY 2u /* node_state_dev (or ghost_tile_dev in the 3D
                                     mode) already holds this call's Uk: skip
                                     making it                                */
#define HYDRO_FLAG_CFL_NEXT 4u    /* also leave the CFL minimum of Uout,
                                     min over cells of dx / (max|v| + c), in
                                     dt_dev[1] (dt_dev then holds 2 doubles) */

/*
 * A batch of leaves (Sec. IV-C): host struct, device arrays.
 *  leaf_coord_dev  int32 [n_leaves][4]: level, ix, iy, iz.
 *  nbr_dev         int32 [n_leaves][27]: slot (dz+1)*9+(dy+1)*3+(dx+1) of the
 *                  neighbour in direction (dx,dy,dz); slot 13 is the leaf
 *                  itself.  A leaf index for SAME_LEAF / COARSER_LEAF, a row
 *                  of children_dev for SAME_REFINED.  Periodic wrap is folded
 *                  into the table.
 *  nbr_kind_dev    uint8 [n_leaves][27]: HYDRO_SAME_LEAF / _SAME_REFINED /
 *                  _COARSER_LEAF.
 *  children_dev    int32 [n_nodes][8]: child leaf at (2x+a, 2y+b, 2z+c) in
 *                  entry c*4+b*2+a, or -1 (children the 3-layer halo never
 *                  reads may be -1).
 *  status_dev      int32, or NULL: kernels OR status bits into it.
 * The tree must be 2:1 balanced over all 26 neighbours ("properly nested").
 */
#define HYDRO_MAX_LEAVES 1048575

typedef struct hydro_grid {
  int32_t n_leaves;
  int32_t n_nodes;
  int32_t n_fields;
  int32_t dtype;
  int32_t base;           /* level-0 sub-grids per axis */
  int32_t reconstruction; /* HYDRO_RECON_AXIS (0) or HYDRO_RECON_3D (1) */
  const int32_t* leaf_coord_dev;
  const int32_t* nbr_dev;
  const uint8_t* nbr_kind_dev;
  const int32_t* children_dev;
  int32_t* status_dev;
  double gamma;            /* ratio of specific heats, e.g. 5.0/3.0        */
  double dual_energy_eta1; /* internal energy from tau when e < eta1 E;
                              <= 0 disables the switch                       */
  /* Coarse-fine flux correction (Sec. V-B-1: fluxes are corrected on
   * coarse-fine boundaries).  Optional: flux_reg_dev == NULL disables it.
   * Tables from hydro_build_reflux; face orientation o = 2*axis + side.
   *  face_slot_dev  int32 [n_leaves][6]: register slot of a coarse face whose
   *                 neighbour is refined, or -1.
   *  fine_slot_dev  int32 [n_leaves][6]: for a face whose neighbour is
   *                 coarser, (slot << 2) | quadrant of the coarse face this
   *                 fine face covers, or -1.
   *  slot_leaf_dev  int32 [n_slots]: coarse leaf of each slot.
   *  orient_begin   host int32 [7]: slots of orientation o are
   *                 [orient_begin[o], orient_begin[o+1]).
   *  flux_reg_dev   double [n_slots][n_fields][320]: caller-owned scratch
   *                 (64 coarse fluxes, then the 16x16 fine fluxes). */
  int32_t n_slots;
  int32_t orient_begin[7];
  const int32_t* face_slot_dev;
  const int32_t* fine_slot_dev;
  const int32_t* slot_leaf_dev;
  double* flux_reg_dev;
  /* Rotating frame (Sec. IV-C: the grid rotates with the binary's initial
   * orbital frequency): angular velocity about the z axis through
   * (0.5, 0.5).  0 = inertial frame.  Non-zero adds to L, per cell from Uk:
   *   s_x: 2 omega s_y + rho omega^2 (x - 0.5)
   *   s_y: rho omega^2 (y - 0.5) - 2 omega s_x
   *   s_z: 0
   *   E:   omega^2 (s_x (x - 0.5) + s_y (y - 0.5))                          */
  double omega;
  /* Restricted copies of the refined blocks: caller-owned device scratch of
   * n_fields * n_nodes * 512 elements of `dtype`, laid out
   * [n_fields][n_nodes][8][8][8]; required when n_nodes > 0, ignored
   * otherwise.  Every substep first writes the coarse (8-cell mean) copy of
   * each refined node of its input state here, then reads the ghost cells
   * of refined face neighbours from it.  Two calls that run at the same
   * time need two buffers. */
  void* node_state_dev;
  /* Materialised ghosted tiles for reconstruction = HYDRO_RECON_3D:
   * caller-owned device scratch of n_fields * n_leaves * 14^3 elements of
   * `dtype`, laid out like the output of hydro_fill_ghosts; required in that
   * mode, ignored otherwise.  Every 3D substep fills it from its Uk. */
  void* ghost_tile_dev;
  /* Chained time steps (Sec. V-B-1: a substep takes part in computing the
   * global time-step size): nonzero makes hydro_rk3_step and its graph take
   * dt_dev as 2 doubles, read dt_dev[1] = the CFL minimum of Un (min over
   * cells of dx / (max|v| + c)) that the previous step left there or that
   * hydro_cfl_dt(grid, Un, 0.0, dt_dev + 1) made, set dt_dev[0] = cfl *
   * dt_dev[1] (cfl > 0), and leave the minimum of Unext in dt_dev[1].  The
   * last substep's kernel takes that minimum from the values it stores, so
   * no pass over Un is needed (with the flux correction or the 3D
   * reconstruction a pass over Unext does it).  The time steps are the same
   * bits as with 0. */
  int32_t cfl_epilogue;
  /* Restricted copies made by the substeps themselves (Sec. VI: no separate
   * buffers of ghost data): with a second caller-owned node buffer of
   * node_state_dev's size and layout, and leaf_node_dev (int32 [n_leaves]:
   * node * 8 + octant of each leaf that is a child of a refined node, else
   * -1; from hydro_build_leaf_node), an RK3 step makes the node copies of Un
   * in a pass and the first two substeps leave those of their outputs as
   * they store them, so the other substeps need no pass.  Ignored with the
   * flux correction or the 3D reconstruction.  Both NULL: a pass before
   * every substep.  Same bits either way. */
  void* node_state2_dev;
  const int32_t* leaf_node_dev;
} hydro_grid;

/*
 * Flux-register tables of a leaf list for the coarse-fine flux correction,
 * on the host, from the outputs of hydro_build_table: face_slot and
 * fine_slot [n_leaves][6], slot_leaf [max_slots], orient_begin [7] (all
 * host, caller-owned).  A coarse leaf owns one slot per face that borders a
 * refined block; slots are numbered by orientation, then leaf.  Returns
 * HYDRO_E_TABLE if a fine face has no matching coarse face.  Synchronous,
 * host only.
 */
int hydro_build_reflux(int32_t n_leaves, const int32_t* leaf_coord, const int32_t* nbr,
                       const uint8_t* kind, int32_t* face_slot, int32_t* fine_slot,
                       int32_t* slot_leaf, int32_t max_slots, int32_t* orient_begin,
                       int32_t* n_slots_out);

/*
 * Neighbour table of a leaf list (Sec. IV-C octree), on the host.
 * leaf_coord: host int32 [n_leaves][4]; outputs nbr [n_leaves][27],
 * kind [n_leaves][27] and children [max_nodes][8] (host, caller-owned).
 * Refined nodes are numbered in order of first reference (leaves ascending,
 * slots ascending).  Returns HYDRO_E_TABLE for duplicate leaves, a leaf that
 * two levels separate from a neighbour, or more than max_nodes refined
 * neighbours.  Synchronous, host only; touches no GPU.
 */
int hydro_build_table(int32_t n_leaves, int32_t base, const int32_t* leaf_coord,
                      int32_t* nbr, uint8_t* kind, int32_t* children,
                      int32_t max_nodes, int32_t* n_nodes_out);

/*
 * For each leaf, node * 8 + octant if it is child `octant` of a row of the
 * children table (children[node][octant] == leaf), else -1; host arrays,
 * children [n_nodes][8] in, leaf_node [n_leaves] out.  Returns HYDRO_E_TABLE
 * if a leaf id is out of range or a leaf is listed twice.  Host only.
 */
int hydro_build_leaf_node(int32_t n_leaves, int32_t n_nodes, const int32_t* children,
                          int32_t* leaf_node);

/*
 * Ghost fill (Sec. VI: neighbours read directly, no message buffers): writes
 * every cell of the ghosted tiles G_dev [nf][n][14][14][14] from U_dev
 * [nf][n][8][8][8] -- interior copy, same-level copy, injection from a
 * coarser leaf, or the mean of 8 finer cells, summed as
 * ((v000+v100)+(v010+v110)) + ((v001+v101)+(v011+v111)) times 0.125.
 * Bit-exact integer/index work; G_dev must not overlap U_dev.
 */
int hydro_fill_ghosts(const hydro_grid* grid, const void* U_dev, void* G_dev, void* stream);

/*
 * One Runge-Kutta substep over all leaves (Sec. V-B-1, compute_fluxes):
 * t = Uk + dt * L(Uk) with L the negative flux divergence from PPM face
 * states and the Kurganov-Tadmor flux, then
 *   Uout = t                       if U0_dev == NULL,
 *   Uout = U0 + beta * (t - U0)    otherwise.
 * The ghost fill is fused: each sub-grid reads its neighbours' cells
 * directly.  dt is read on the device from *dt_dev (binary64).
 * With flux-register tables in the grid, the fluxes through coarse-fine
 * faces are recorded and then corrected: each coarse cell next to a refined
 * face gets q = (Havg - Hc)/dx with Havg = 0.25((H00 + H10) + (H01 + H11))
 * of the 4 fine fluxes and Hc its own, and Uout -= w dt q on its high face,
 * += on its low face (w = 1 without U0, else beta; faces x, y, z, low first).
 * Before the fluxes, the restricted copies of the refined nodes are made
 * from Uk into grid->node_state_dev (when the tree has refined nodes), or,
 * with reconstruction HYDRO_RECON_3D, the ghosted tiles of Uk into
 * grid->ghost_tile_dev.  Uout_dev may alias neither Uk_dev nor U0_dev.
 * flags: HYDRO_FLAG_VALIDATE; HYDRO_FLAG_NODES_READY when that scratch was
 * made from this Uk by an earlier call and not overwritten since (the
 * caller's promise: it is not checked).
 */
int hydro_step(const hydro_grid* grid, const void* U0_dev, const void* Uk_dev, void* Uout_dev,
               const double* dt_dev, double beta, uint32_t flags, void* stream);

/*
 * Same substep, launched once per leaf round-robin over a pool of n_streams
 * HIP streams owned by the library (the paper's one-kernel-per-sub-grid
 * design with a pool of 128 streams, Sec. IV-C).  Ordered after earlier work
 * on `stream`, and later work on `stream` waits for all of it.  For
 * comparison with hydro_step; results are bit-identical to it.
 */
int hydro_step_per_leaf(const hydro_grid* grid, const void* U0_dev, const void* Uk_dev,
                        void* Uout_dev, const double* dt_dev, double beta, int32_t n_streams,
                        void* stream);

/*
 * Global time-step size (Sec. V-B-1): *dt_dev = cfl * min over all leaves and
 * interior cells of dx_L / (max(|v_x|,|v_y|,|v_z|) + c), in binary64 for
 * either dtype.  Exact min reduction: the result does not depend on order.
 * cfl == 0 leaves the minimum itself (the input of a chained RK3 step).
 */
int hydro_cfl_dt(const hydro_grid* grid, const void* U_dev, double cfl, double* dt_dev,
                 void* stream);

/*
 * Conserved totals: totals_dev[f] = sum over cells of U_f * dx_L^3, binary64
 * with double-double (TwoSum) accumulation.  Uses a library-owned scratch
 * buffer (allocated on first use per device, grown with hipMalloc when a
 * larger grid needs more) that every call on that device shares: calls
 * that overlap in time on one device (two streams, or two host threads)
 * race on it and must be ordered by the caller.
 */
int hydro_totals(const hydro_grid* grid, const void* U_dev, double* totals_dev, void* stream);

/*
 * The same totals for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): same
 * kernels and summation order, so the same bits as hydro_totals.  Its
 * partial sums live in a fixed array inside the library (256 KiB per GPU,
 * room for every grid hydro_totals accepts; a larger request returns
 * HYDRO_E_ARG), held until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call.  The array's device address is looked
 * up on the first call on each device.  Every call overwrites the partial
 * sums it reads, so nothing needs clearing between calls, but all calls on
 * one GPU share the array: calls that overlap in time on one device race.
 */
int hydro_totals_noalloc(const hydro_grid* grid, const void* U_dev, double* totals_dev,
                         void* stream);

/*
 * One SSP-RK3 time step (three substeps, Sec. I):
 *   if cfl > 0: *dt_dev = hydro_cfl_dt(Un);  else *dt_dev is used as given;
 *   W1 = Un + dt L(Un);  W2 = Un + 1/4 (W1 + dt L(W1) - Un);
 *   Unext = Un + 2/3 (W2 + dt L(W2) - Un).
 * W1_dev, W2_dev are caller scratch of the state's size; Unext_dev may be
 * W1_dev but not Un_dev or W2_dev.
 */
int hydro_rk3_step(const hydro_grid* grid, const void* Un_dev, void* W1_dev, void* W2_dev,
                   void* Unext_dev, double cfl, double* dt_dev, void* stream);

/*
 * The same RK3 step captured once into a HIP graph (argument values and
 * pointers are frozen at capture).  hydro_graph_launch replays it on
 * `stream`; hydro_graph_destroy frees it.  *graph_out is an opaque handle.
 */
int hydro_rk3_graph_create(const hydro_grid* grid, const void* Un_dev, void* W1_dev,
                           void* W2_dev, void* Unext_dev, double cfl, double* dt_dev,
                           void** graph_out);
int hydro_graph_launch(void* graph, void* stream);
int hydro_graph_destroy(void* graph);

/*
 * Waits for `stream`, then reads grid->status_dev: returns HYDRO_OK,
 * HYDRO_E_UNPHYSICAL or HYDRO_E_TABLE.  Synchronous.
 */
int hydro_check_status(const hydro_grid* grid, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* hydro_last_error(void);

/*
 * Launch options of the fused substep kernel for one (dtype, n_fields) pair;
 * the defaults are 1 wave per SIMD and the XCD remap on.  The autotuner
 * (paper_2210_06437_amd/autotune.py) times the choices and records the
 * fastest; the Python binding applies its recorded choices at import.
 *   HYDRO_OPT_WAVES_PER_SIMD  1 or 2: register budget of the kernel (2 waves
 *                             per SIMD caps it at 256 VGPRs, which may spill)
 *   HYDRO_OPT_XCD_REMAP       which leaves each of the 8 XCDs works on:
 *                             0 in launch order, 1 one contiguous range per
 *                             XCD, c (a power of two in [2, 4096]) chunks
 *                             of c consecutive leaves dealt in turn
 *   HYDRO_OPT_WAVES_PER_LEAF  1 or 2: wavefronts per leaf; with 2 (n_fields
 *                             > 6 only) the second wavefront of each leaf
 *                             evolves the passive species, taking each face's
 *                             velocities and signal speed from the first
 *                             through LDS (same bits, half the registers)
 *   HYDRO_OPT_CFL_EPILOGUE    1 or 0: where a step that leaves the CFL
 *                             minimum of its output (HYDRO_FLAG_CFL_NEXT,
 *                             chained RK3 steps) takes it: in the substep
 *                             kernel itself, or in a pass over the output
 *   HYDRO_OPT_FUSED_RESTRICT  1 or 0: whether an RK3 step with
 *                             node_state2_dev lets its substeps leave the
 *                             node copies of their outputs (1) or makes
 *                             them in a pass before each substep (0)
 *   HYDRO_OPT_3D_WORKGROUP    0, 1 or 2: the 3D step with one wavefront
 *                             per leaf (0) or one 256-thread workgroup per
 *                             leaf where its face fluxes fit in LDS
 *                             (binary64 up to 11 fields, binary32 up to
 *                             16): evaluating each face from both sides'
 *                             line parabolas (1), or reconstructing each
 *                             (cell, line) once per face orientation, the
 *                             lines common to the x- and y-faces once for
 *                             both, and using both ends of its parabola
 *                             (2, the default)
 * Every choice computes the same bits.  Options are process-wide and take effect at the next launch (a captured
 * graph keeps the kernel it was captured with).  Host only, thread-safe.
 */
#define HYDRO_OPT_WAVES_PER_SIMD 1
#define HYDRO_OPT_XCD_REMAP 2
#define HYDRO_OPT_WAVES_PER_LEAF 3
#define HYDRO_OPT_CFL_EPILOGUE 4
#define HYDRO_OPT_FUSED_RESTRICT 5
#define HYDRO_OPT_3D_WORKGROUP 6
int hydro_set_option(int32_t dtype, int32_t n_fields, int32_t option, int32_t value);
int hydro_get_option(int32_t dtype, int32_t n_fields, int32_t option, int32_t* value);

/* Library version, major*10000 + minor*100 + patch. */
int hydro_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OCTOHYDRO_H */
