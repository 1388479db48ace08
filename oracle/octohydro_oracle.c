/*
 * octohydro_oracle.c -- plain, slow FP64 CPU oracle for the octree hydro step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load it.
 * It shares no code, header, table or constant generator with the HIP library.
 *
 * What it computes (paper: "Distributed, combined CPU and GPU profiling within
 * HPX using APEX", arXiv 2210.06437):
 *   - the octree of 8^3 sub-grids, each refinable into 8 children at twice the
 *     resolution, properly nested (Sec. IV-C);
 *   - the ghost-cell fill of every sub-grid from its neighbours, done as a
 *     direct read of neighbour memory rather than messages (Sec. VI);
 *   - PPM reconstruction of the evolved variables (Sec. V-B-1, kernel
 *     "reconstruct"), the central-scheme fluxes of Kurganov & Tadmor for the
 *     inviscid Euler equations (Sec. IV-C, kernel "flux" in Sec. V-B-1), the
 *     flux-divergence update and the global time-step size of one
 *     Runge-Kutta substep (Sec. V-B-1, task compute_fluxes); three hydro
 *     substeps per time step (Sec. I).
 * The paper names these methods without equations, so every formula below is
 * the textbook form of the named method, written in the order the method
 * states it:
 *   PPM: Colella & Woodward (1984), uniform grid, no flattening/steepening,
 *        applied to each conserved field separately;
 *   flux: Kurganov & Tadmor (2000) semi-discrete central flux evaluated at the
 *        face centre;
 *   time: Shu & Osher (1988) SSP-RK3;
 *   EOS: ideal gas with an entropy tracer tau = (rho e)^(1/gamma) used by a
 *        dual-energy switch (Bryan et al. 1995 style).
 * Compile with -O2 -ffp-contract=off and no fast-math: every operation below
 * is one IEEE-754 binary64 operation, rounded once, in the order written.
 *
 * Layouts: U[nf][n_leaves][8][8][8] (x fastest); ghosted tile
 * G[nf][n_leaves][14][14][14]; interior of a tile at [3,11)^3.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "octohydro_oracle.h"

#define SUB 8            /* sub-grid edge N (Sec. IV-C: usually N = 8)      */
#define GH 3             /* ghost layers needed by the PPM stencil          */
#define TW 14            /* tile width SUB + 2*GH                           */
#define TILE (TW * TW * TW)
#define CELLS (SUB * SUB * SUB)

/* ------------------------------------------------------------------------ */
/* Octree leaf lookup: sorted keys + binary search.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t level, x, y, z;
  int32_t idx;
} okey;

static int okey_cmp(const void* pa, const void* pb) {
  const okey* a = (const okey*)pa;
  const okey* b = (const okey*)pb;
  if (a->level != b->level) return a->level < b->level ? -1 : 1;
  if (a->z != b->z) return a->z < b->z ? -1 : 1;
  if (a->y != b->y) return a->y < b->y ? -1 : 1;
  if (a->x != b->x) return a->x < b->x ? -1 : 1;
  return 0;
}

static int32_t find_leaf(const okey* keys, int n, int32_t level, int32_t x, int32_t y,
                         int32_t z) {
  okey probe = {level, x, y, z, -1};
  const okey* hit = (const okey*)bsearch(&probe, keys, (size_t)n, sizeof(okey), okey_cmp);
  return hit ? hit->idx : -1;
}

static int32_t wrapi(int32_t g, int32_t m) {
  int32_t r = g % m;
  return r < 0 ? r + m : r;
}

/* Refined nodes get ids in order of first reference (leaves ascending, then
 * slots ascending).  A tiny open-addressing map finds the id of a node. */
typedef struct {
  int64_t* key;
  int32_t* val;
  int64_t cap;
} omap;

static int64_t node_key(int32_t level, int32_t x, int32_t y, int32_t z) {
  return ((int64_t)level << 54) | ((int64_t)z << 36) | ((int64_t)y << 18) | (int64_t)x;
}

static int32_t omap_get_or_add(omap* m, int64_t k, int32_t next_id, int* added) {
  uint64_t h = (uint64_t)k * 0x9E3779B97F4A7C15ull;
  int64_t i = (int64_t)(h % (uint64_t)m->cap);
  for (;;) {
    if (m->key[i] == -1) {
      m->key[i] = k;
      m->val[i] = next_id;
      *added = 1;
      return next_id;
    }
    if (m->key[i] == k) {
      *added = 0;
      return m->val[i];
    }
    i = (i + 1) % m->cap;
  }
}

int oracle_build_table(int32_t n_leaves, int32_t base, const int32_t* leaf_coord,
                       int32_t* nbr, uint8_t* kind, int32_t* children, int32_t max_nodes,
                       int32_t* n_nodes_out) {
  if (n_leaves <= 0 || base <= 0) return ORACLE_E_ARG;
  okey* keys = (okey*)malloc(sizeof(okey) * (size_t)n_leaves);
  for (int32_t i = 0; i < n_leaves; ++i) {
    keys[i].level = leaf_coord[4 * i + 0];
    keys[i].x = leaf_coord[4 * i + 1];
    keys[i].y = leaf_coord[4 * i + 2];
    keys[i].z = leaf_coord[4 * i + 3];
    keys[i].idx = i;
  }
  qsort(keys, (size_t)n_leaves, sizeof(okey), okey_cmp);
  for (int32_t i = 1; i < n_leaves; ++i)
    if (okey_cmp(&keys[i - 1], &keys[i]) == 0) {
      free(keys);
      return ORACLE_E_TABLE; /* duplicate leaf */
    }

  omap map;
  map.cap = 4 * (int64_t)n_leaves + 64;
  map.key = (int64_t*)malloc(sizeof(int64_t) * (size_t)map.cap);
  map.val = (int32_t*)malloc(sizeof(int32_t) * (size_t)map.cap);
  for (int64_t i = 0; i < map.cap; ++i) map.key[i] = -1;

  int status = ORACLE_OK;
  int32_t n_nodes = 0;
  for (int32_t n = 0; n < n_leaves && status == ORACLE_OK; ++n) {
    const int32_t L = leaf_coord[4 * n + 0];
    const int32_t c[3] = {leaf_coord[4 * n + 1], leaf_coord[4 * n + 2], leaf_coord[4 * n + 3]};
    const int32_t blocks = base << L; /* sub-grids per axis at level L */
    for (int32_t dz = -1; dz <= 1 && status == ORACLE_OK; ++dz)
      for (int32_t dy = -1; dy <= 1 && status == ORACLE_OK; ++dy)
        for (int32_t dx = -1; dx <= 1; ++dx) {
          const int32_t slot = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          const int32_t t[3] = {wrapi(c[0] + dx, blocks), wrapi(c[1] + dy, blocks),
                                wrapi(c[2] + dz, blocks)};
          int32_t m = find_leaf(keys, n_leaves, L, t[0], t[1], t[2]);
          if (m >= 0) {
            nbr[27 * n + slot] = m;
            kind[27 * n + slot] = ORACLE_SAME_LEAF;
            continue;
          }
          if (L > 0) {
            m = find_leaf(keys, n_leaves, L - 1, t[0] >> 1, t[1] >> 1, t[2] >> 1);
            if (m >= 0) {
              nbr[27 * n + slot] = m;
              kind[27 * n + slot] = ORACLE_COARSER_LEAF;
              continue;
            }
          }
          /* The neighbour block is refined: the children that the 3-layer
           * halo touches must be leaves one level finer. */
          int added = 0;
          const int32_t id = omap_get_or_add(&map, node_key(L, t[0], t[1], t[2]), n_nodes, &added);
          if (added) {
            if (n_nodes >= max_nodes) {
              status = ORACLE_E_TABLE;
              break;
            }
            for (int32_t q = 0; q < 8; ++q)
              children[8 * id + q] = find_leaf(keys, n_leaves, L + 1, 2 * t[0] + (q & 1),
                                               2 * t[1] + ((q >> 1) & 1), 2 * t[2] + (q >> 2));
            ++n_nodes;
          }
          const int32_t d[3] = {dx, dy, dz};
          for (int32_t q = 0; q < 8; ++q) {
            const int32_t a[3] = {q & 1, (q >> 1) & 1, q >> 2};
            int needed = 1;
            for (int k = 0; k < 3; ++k)
              if ((d[k] == -1 && a[k] != 1) || (d[k] == 1 && a[k] != 0)) needed = 0;
            if (needed && children[8 * id + q] < 0) status = ORACLE_E_TABLE;
          }
          nbr[27 * n + slot] = id;
          kind[27 * n + slot] = ORACLE_SAME_REFINED;
        }
  }
  free(map.key);
  free(map.val);
  free(keys);
  *n_nodes_out = n_nodes;
  return status;
}

/* ------------------------------------------------------------------------ */
/* Ghost fill (Sec. VI: ghost cells read directly from neighbour memory).   */
/* ------------------------------------------------------------------------ */

static double uval(const ogrid* g, const double* U, int f, int32_t leaf, int32_t lx, int32_t ly,
                   int32_t lz) {
  return U[((size_t)f * g->n_leaves + leaf) * CELLS + (size_t)(lz * 64 + ly * 8 + lx)];
}

/* Value of tile cell (tx,ty,tz) of `leaf`, field f: interior copy, or the
 * neighbour value by same-level copy, injection from a coarser leaf, or the
 * mean of the 8 covering cells of a finer leaf. */
static double tile_value(const ogrid* g, const double* U, int f, int32_t leaf, int32_t tx,
                         int32_t ty, int32_t tz) {
  const int32_t t[3] = {tx, ty, tz};
  int32_t r[3];
  for (int k = 0; k < 3; ++k) r[k] = t[k] < GH ? -1 : (t[k] >= GH + SUB ? 1 : 0);
  const int32_t slot = (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
  if (slot == 13) return uval(g, U, f, leaf, tx - GH, ty - GH, tz - GH);

  const int32_t L = g->coord[4 * leaf + 0];
  const int32_t ncell = SUB * (g->base << L); /* cells per axis at level L */
  int32_t gi[3];
  for (int k = 0; k < 3; ++k) gi[k] = wrapi(SUB * g->coord[4 * leaf + 1 + k] + t[k] - GH, ncell);
  const int32_t m = g->nbr[27 * leaf + slot];
  const int kd = g->kind[27 * leaf + slot];
  if (kd == ORACLE_SAME_LEAF) {
    int32_t l[3];
    for (int k = 0; k < 3; ++k) l[k] = gi[k] - SUB * g->coord[4 * m + 1 + k];
    return uval(g, U, f, m, l[0], l[1], l[2]);
  }
  if (kd == ORACLE_COARSER_LEAF) {
    int32_t l[3];
    for (int k = 0; k < 3; ++k) l[k] = (gi[k] >> 1) - SUB * g->coord[4 * m + 1 + k];
    return uval(g, U, f, m, l[0], l[1], l[2]);
  }
  /* SAME_REFINED: m indexes the children table. */
  int32_t lc[3], ch[3];
  for (int k = 0; k < 3; ++k) {
    lc[k] = gi[k] & (SUB - 1); /* coarse cell within the refined block */
    ch[k] = lc[k] >> 2;        /* which child covers it */
  }
  const int32_t child = g->children[8 * m + ch[2] * 4 + ch[1] * 2 + ch[0]];
  double v[2][2][2];
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        v[a][b][c] = uval(g, U, f, child, (2 * lc[0] + a) & 7, (2 * lc[1] + b) & 7,
                          (2 * lc[2] + c) & 7);
  return 0.125 * (((v[0][0][0] + v[1][0][0]) + (v[0][1][0] + v[1][1][0])) +
                  ((v[0][0][1] + v[1][0][1]) + (v[0][1][1] + v[1][1][1])));
}

void oracle_fill_ghosts(const ogrid* g, const double* U, double* G) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t n = 0; n < g->n_leaves; ++n)
    for (int f = 0; f < g->nf; ++f) {
      double* T = G + ((size_t)f * g->n_leaves + n) * TILE;
      for (int32_t tz = 0; tz < TW; ++tz)
        for (int32_t ty = 0; ty < TW; ++ty)
          for (int32_t tx = 0; tx < TW; ++tx)
            T[(tz * TW + ty) * TW + tx] = tile_value(g, U, f, n, tx, ty, tz);
    }
}

/* ------------------------------------------------------------------------ */
/* PPM reconstruction along one pencil (Colella & Woodward 1984).           */
/* ------------------------------------------------------------------------ */

/* Input q[0..n); output, for cells j in [2, n-2), the left and right face
 * values qL[j] (at j-1/2) and qR[j] (at j+1/2) after monotonisation.
 * Entries outside [2, n-2) are left untouched. */
void oracle_ppm_1d(const double* q, int n, double* qL, double* qR) {
  double dm[64], qf[64];
  if (n > 64 || n < 5) return;
  /* Limited slope of each cell (CW84 eq. 1.8). */
  for (int j = 1; j < n - 1; ++j) {
    const double dq = 0.5 * (q[j + 1] - q[j - 1]);
    const double dl = q[j] - q[j - 1];
    const double dr = q[j + 1] - q[j];
    if (dl * dr > 0.0) {
      const double lim = fmin(fabs(dq), fmin(2.0 * fabs(dl), 2.0 * fabs(dr)));
      dm[j] = copysign(lim, dq);
    } else {
      dm[j] = 0.0;
    }
  }
  /* Interface value at j+1/2 (CW84 eq. 1.6 on a uniform grid). */
  for (int j = 1; j < n - 2; ++j)
    qf[j] = 0.5 * (q[j] + q[j + 1]) - (dm[j + 1] - dm[j]) * (1.0 / 6.0);
  /* Monotonisation of the parabola in each cell (CW84 eq. 1.10). */
  for (int j = 2; j < n - 2; ++j) {
    double l = qf[j - 1], r = qf[j];
    const double c = q[j];
    if ((r - c) * (c - l) <= 0.0) {
      l = c;
      r = c;
    } else {
      const double dlr = r - l;
      const double a6 = 6.0 * (c - 0.5 * (l + r));
      if (dlr * a6 > dlr * dlr)
        l = 3.0 * c - 2.0 * r;
      else if (-(dlr * dlr) > dlr * a6)
        r = 3.0 * c - 2.0 * l;
    }
    qL[j] = l;
    qR[j] = r;
  }
}

/* ------------------------------------------------------------------------ */
/* Ideal-gas EOS with dual-energy switch, and the KT face flux.             */
/* ------------------------------------------------------------------------ */

/* Primitive quantities of a conserved state u = (rho, sx, sy, sz, E, tau, ...).
 * Returns 1 if the state is unphysical (rho <= 0 or p <= 0). */
static int eos(const double* u, double gamma, double eta1, double* rinv, double* p, double* c) {
  const double rho = u[0];
  *rinv = 1.0 / rho;
  const double ss = (u[1] * u[1] + u[2] * u[2]) + u[3] * u[3];
  double ei = u[4] - 0.5 * ss * (*rinv);
  if (ei < eta1 * u[4]) ei = pow(u[5], gamma); /* internal energy from tau */
  *p = (gamma - 1.0) * ei;
  *c = sqrt(gamma * (*p) * (*rinv));
  return !(rho > 0.0) || !(*p > 0.0);
}

/* Physical flux of state u along direction d (0,1,2) given v_n and p. */
static void phys_flux(int d, int nf, const double* u, double vn, double p, double* F) {
  F[0] = u[1 + d];
  for (int m = 0; m < 3; ++m) F[1 + m] = u[1 + m] * vn;
  F[1 + d] = F[1 + d] + p;
  F[4] = (u[4] + p) * vn;
  for (int k = 5; k < nf; ++k) F[k] = u[k] * vn;
}

/* Kurganov-Tadmor central flux at one face, left state UL, right state UR.
 * Returns the number of unphysical states seen (0..2). */
int oracle_face_flux(int d, int nf, const double* UL, const double* UR, double gamma,
                     double eta1, double* H) {
  double riL, pL, cL, riR, pR, cR, FL[ORACLE_MAX_NF], FR[ORACLE_MAX_NF];
  int bad = eos(UL, gamma, eta1, &riL, &pL, &cL);
  bad += eos(UR, gamma, eta1, &riR, &pR, &cR);
  const double vL = UL[1 + d] * riL;
  const double vR = UR[1 + d] * riR;
  const double a = fmax(fabs(vL) + cL, fabs(vR) + cR);
  phys_flux(d, nf, UL, vL, pL, FL);
  phys_flux(d, nf, UR, vR, pR, FR);
  const double ha = 0.5 * a;
  for (int k = 0; k < nf; ++k) H[k] = 0.5 * (FL[k] + FR[k]) - ha * (UR[k] - UL[k]);
  return bad;
}

/* ------------------------------------------------------------------------ */
/* One Runge-Kutta substep over all leaves.                                 */
/* ------------------------------------------------------------------------ */

/* Shu-Osher stage: t = Uk + dt L; the first stage keeps t, the later ones
 * take the convex combination (1 - beta) U0 + beta t written as
 * U0 + beta (t - U0), which leaves a steady state exactly unchanged. */
static void combine(int has_u0, double beta, double dt, double u0, double uk, double lrate,
                    double* out) {
  const double t = uk + dt * lrate;
  *out = has_u0 ? u0 + beta * (t - u0) : t;
}

/* Source of field f (1..4: s_x, s_y, s_z, E) in a frame rotating with
 * angular velocity omega about the z axis through (0.5, 0.5) (Sec. IV-C: the
 * grid rotates with the binary's initial orbital frequency): Coriolis
 * -2 Omega x s and centrifugal rho Omega^2 r_perp on the momentum, and the
 * centrifugal force's work Omega^2 (s . r_perp) on the energy; the Coriolis
 * force does no work.  Evaluated from the cell values of Uk at the cell
 * centre. */
static double rotating_source(const ogrid* g, const double* Uk, int32_t n, int32_t cell, int f) {
  const int32_t L = g->coord[4 * n + 0];
  const double dx = 1.0 / (double)(SUB * (g->base << L));
  const int32_t i = cell & 7, j = (cell >> 3) & 7;
  const double rx = ((double)(SUB * g->coord[4 * n + 1] + i) + 0.5) * dx - 0.5;
  const double ry = ((double)(SUB * g->coord[4 * n + 2] + j) + 0.5) * dx - 0.5;
  const size_t fs = (size_t)g->n_leaves * CELLS;
  const size_t at = (size_t)n * CELLS + cell;
  const double rho = Uk[at], sx = Uk[fs + at], sy = Uk[2 * fs + at];
  const double om2 = g->omega * g->omega;
  const double tw = 2.0 * g->omega;
  switch (f) {
    case 1: return tw * sy + rho * om2 * rx;
    case 2: return rho * om2 * ry - tw * sx;
    case 4: return om2 * (sx * rx + sy * ry);
    default: return 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* Full three-dimensional reconstruction and face quadrature (Sec. V-B-1:    */
/* the reconstruct kernel does a full 3D reconstruction, the flux kernel     */
/* integrates the face fluxes by quadrature).                                */
/* ------------------------------------------------------------------------ */

/* Value of one field (tile Tf) of tile cell t at the point t + p/2, p in
 * {-1,0,1}^3 \ {0}: a face centre, edge midpoint or corner of the cell.  It
 * comes from the same PPM as along an axis, applied to the line of cells
 * t + m e, m = -2..2, where e is p or -p, whichever has its first non-zero
 * component positive (13 lines through each cell).  The point is the right
 * end (+e/2) of the cell's monotonised parabola when e = p, the left end
 * otherwise. */
double oracle_point_value(const double* Tf, const int32_t t[3], const int32_t p[3]) {
  const int32_t first = p[0] != 0 ? p[0] : (p[1] != 0 ? p[1] : p[2]);
  const int right = first > 0;
  const int32_t e[3] = {right ? p[0] : -p[0], right ? p[1] : -p[1], right ? p[2] : -p[2]};
  double q[5], qL[5], qR[5];
  for (int32_t m = -2; m <= 2; ++m)
    q[m + 2] = Tf[((t[2] + m * e[2]) * TW + (t[1] + m * e[1])) * TW + (t[0] + m * e[0])];
  oracle_ppm_1d(q, 5, qL, qR);
  return right ? qR[2] : qL[2];
}

/* Flux through the face normal to d between tile cells tl and tl + d: the
 * Kurganov-Tadmor flux at its 9 points (pu, pv) in {-1,0,1}^2 (u < v the
 * other two axes), the left state from cell tl at offset (+1, pu, pv)/2 and
 * the right state from cell tl + d at offset (-1, pu, pv)/2, combined by the
 * tensor-product Simpson rule, weights 1 (corners), 4 (edge midpoints) and
 * 16 (centre) over 36, summed as
 *   ((corners + 4 edges) + 16 centre) / 36,
 *   corners = (H(-1,-1) + H(1,1)) + (H(1,-1) + H(-1,1)),
 *   edges   = (H(0,-1) + H(0,1)) + (H(-1,0) + H(1,0)),
 * an order that a mirror of either transverse axis only commutes.  Returns
 * the number of unphysical states seen. */
int oracle_face_flux_3d(const ogrid* g, const double* T, int d, const int32_t tl[3],
                        double* H) {
  const int nf = g->nf;
  const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;
  int32_t tr[3] = {tl[0], tl[1], tl[2]};
  tr[d] += 1;
  double Hp[3][3][ORACLE_MAX_NF]; /* [pv + 1][pu + 1][field] */
  double UL[ORACLE_MAX_NF], UR[ORACLE_MAX_NF];
  int bad = 0;
  for (int32_t pv = -1; pv <= 1; ++pv)
    for (int32_t pu = -1; pu <= 1; ++pu) {
      int32_t pl[3], pr[3];
      pl[d] = 1;
      pr[d] = -1;
      pl[u] = pr[u] = pu;
      pl[v] = pr[v] = pv;
      for (int f = 0; f < nf; ++f) {
        UL[f] = oracle_point_value(T + (size_t)f * TILE, tl, pl);
        UR[f] = oracle_point_value(T + (size_t)f * TILE, tr, pr);
      }
      bad += oracle_face_flux(d, nf, UL, UR, g->gamma, g->eta1, Hp[pv + 1][pu + 1]);
    }
  for (int f = 0; f < nf; ++f) {
#define HP(a, b) Hp[(b) + 1][(a) + 1][f]
    const double corners = (HP(-1, -1) + HP(1, 1)) + (HP(1, -1) + HP(-1, 1));
    const double edges = (HP(0, -1) + HP(0, 1)) + (HP(-1, 0) + HP(1, 0));
    H[f] = ((corners + 4.0 * edges) + 16.0 * HP(0, 0)) / 36.0;
#undef HP
  }
  return bad;
}

/* Position of transverse cell (u, v) in a face normal to d: u, v are the
 * two other axes in increasing order (d=0: y,z; d=1: x,z; d=2: x,y). */
static int32_t face_index(int32_t u, int32_t v) { return u + SUB * v; }

int64_t oracle_step_subset(const ogrid* g, const double* U0, const double* Uk, double* Uout,
                           double dt, double beta, const int32_t* subset, int32_t n_subset) {
  return oracle_step_record(g, U0, Uk, Uout, dt, beta, subset, n_subset, NULL);
}

int64_t oracle_step_record(const ogrid* g, const double* U0, const double* Uk, double* Uout,
                           double dt, double beta, const int32_t* subset, int32_t n_subset,
                           double* face_flux) {
  const int nf = g->nf;
  const int32_t n_work = subset ? n_subset : g->n_leaves;
  int64_t bad_total = 0;
#pragma omp parallel reduction(+ : bad_total)
  {
    double* T = (double*)malloc(sizeof(double) * (size_t)nf * TILE);
    double* dH = (double*)malloc(sizeof(double) * (size_t)nf * 3 * CELLS);
    double pen[ORACLE_MAX_NF][TW], pL[ORACLE_MAX_NF][TW], pR[ORACLE_MAX_NF][TW];
    double UL[ORACLE_MAX_NF], UR[ORACLE_MAX_NF], H[TW][ORACLE_MAX_NF];
#pragma omp for schedule(dynamic, 4)
    for (int32_t w = 0; w < n_work; ++w) {
      const int32_t n = subset ? subset[w] : w;
      const int32_t L = g->coord[4 * n + 0];
      const double inv_dx = (double)(SUB * (g->base << L));
      for (int f = 0; f < nf; ++f)
        for (int32_t tz = 0; tz < TW; ++tz)
          for (int32_t ty = 0; ty < TW; ++ty)
            for (int32_t tx = 0; tx < TW; ++tx)
              T[(size_t)f * TILE + (tz * TW + ty) * TW + tx] = tile_value(g, Uk, f, n, tx, ty, tz);
      /* Flux differences along each direction d for every interior cell. */
      for (int d = 0; d < 3; ++d)
        for (int32_t b = 0; b < SUB; ++b)
          for (int32_t a = 0; a < SUB; ++a) {
            /* pencil along d through interior transverse cell (a, b) */
            for (int f = 0; f < nf; ++f) {
              for (int32_t k = 0; k < TW; ++k) {
                int32_t t[3];
                t[d] = k;
                t[(d + 1) % 3] = a + GH;
                t[(d + 2) % 3] = b + GH;
                pen[f][k] = T[(size_t)f * TILE + (t[2] * TW + t[1]) * TW + t[0]];
              }
              oracle_ppm_1d(pen[f], TW, pL[f], pR[f]);
            }
            /* face k+1/2 between tile cells k and k+1, k = 2..10 */
            for (int32_t k = GH - 1; k < GH + SUB; ++k) {
              if (g->recon == 1) {
                int32_t tl[3];
                tl[d] = k;
                tl[(d + 1) % 3] = a + GH;
                tl[(d + 2) % 3] = b + GH;
                bad_total += oracle_face_flux_3d(g, T, d, tl, H[k]);
                continue;
              }
              for (int f = 0; f < nf; ++f) {
                UL[f] = pR[f][k];
                UR[f] = pL[f][k + 1];
              }
              bad_total += oracle_face_flux(d, nf, UL, UR, g->gamma, g->eta1, H[k]);
            }
            if (face_flux) {
              /* the fluxes through the leaf's two faces normal to d */
              int32_t l[3];
              l[d] = 0;
              l[(d + 1) % 3] = a;
              l[(d + 2) % 3] = b;
              const int32_t u = d == 0 ? l[1] : l[0], v = d == 2 ? l[1] : l[2];
              for (int side = 0; side < 2; ++side)
                for (int f = 0; f < nf; ++f)
                  face_flux[((((size_t)n * 3 + d) * 2 + side) * CELLS / SUB + face_index(u, v)) * nf +
                            f] = H[side ? GH + SUB - 1 : GH - 1][f];
            }
            for (int32_t i = 0; i < SUB; ++i) {
              int32_t l[3];
              l[d] = i;
              l[(d + 1) % 3] = a;
              l[(d + 2) % 3] = b;
              const int32_t cell = l[2] * 64 + l[1] * 8 + l[0];
              for (int f = 0; f < nf; ++f)
                dH[((size_t)f * 3 + d) * CELLS + cell] = H[i + GH][f] - H[i + GH - 1][f];
            }
          }
      for (int f = 0; f < nf; ++f)
        for (int32_t cell = 0; cell < CELLS; ++cell) {
          const double* q = dH + (size_t)f * 3 * CELLS;
          double lrate = -((q[cell] + q[CELLS + cell]) + q[2 * CELLS + cell]) * inv_dx;
          if (g->omega != 0.0 && f >= 1 && f <= 4)
            lrate = lrate + rotating_source(g, Uk, n, cell, f);
          const size_t at = ((size_t)f * g->n_leaves + n) * CELLS + cell;
          combine(U0 != NULL, beta, dt, U0 ? U0[at] : 0.0, Uk[at], lrate, &Uout[at]);
        }
    }
    free(T);
    free(dH);
  }
  return bad_total;
}

int64_t oracle_step(const ogrid* g, const double* U0, const double* Uk, double* Uout, double dt,
                    double beta) {
  return oracle_step_subset(g, U0, Uk, Uout, dt, beta, NULL, 0);
}

/* ------------------------------------------------------------------------ */
/* Coarse-fine flux correction (Sec. V-B-1: compute_fluxes "corrects these   */
/* fluxes on coarse-fine boundaries").                                       */
/* ------------------------------------------------------------------------ */

/* After a substep, each coarse cell next to a refined face neighbour gets the
 * flux through that face replaced by the area-weighted mean of the 4 fine
 * fluxes the refined side computed there,
 *   H_avg = 0.25 * ((H00 + H10) + (H01 + H11))   (first index along u),
 * applied as a correction of the stored result: with q = (H_avg - H_c)/dx,
 * Uout -= w dt q on the coarse cell's high face, += on its low face, where
 * H_c is the flux the coarse leaf used and w = 1 (first stage) or beta.
 * Faces are visited in the order x, y, z and low before high.  face_flux
 * holds the fluxes recorded by oracle_step_record for every leaf involved. */
void oracle_reflux(const ogrid* g, double* Uout, double dt, double w, const double* face_flux,
                   const int32_t* subset, int32_t n_subset) {
  const int nf = g->nf;
  const int32_t n_work = subset ? n_subset : g->n_leaves;
  const double wdt = w * dt;
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t it = 0; it < n_work; ++it) {
    const int32_t c = subset ? subset[it] : it;
    const int32_t L = g->coord[4 * c + 0];
    const double inv_dx = (double)(SUB * (g->base << L));
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side) {
        int32_t r[3] = {0, 0, 0};
        r[d] = side ? 1 : -1;
        const int32_t slot = (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
        if (g->kind[27 * c + slot] != ORACLE_SAME_REFINED) continue;
        const int32_t node = g->nbr[27 * c + slot];
        for (int32_t v = 0; v < SUB; ++v)
          for (int32_t u = 0; u < SUB; ++u) {
            /* the coarse face cell (u, v) is covered by fine faces (2u+i, 2v+j) */
            double Hf[2][2][ORACLE_MAX_NF];
            for (int j = 0; j < 2; ++j)
              for (int i = 0; i < 2; ++i) {
                const int32_t fu = 2 * u + i, fv = 2 * v + j;
                int32_t ch[3];
                ch[d] = side ? 0 : 1; /* children on the near side of the node */
                ch[d == 0 ? 1 : 0] = fu >> 3;
                ch[d == 2 ? 1 : 2] = fv >> 3;
                const int32_t fine = g->children[8 * node + ch[2] * 4 + ch[1] * 2 + ch[0]];
                /* the fine leaf's face on the coarse side: its low face when the
                 * coarse cell lies below it, else its high face */
                const int fside = side ? 0 : 1;
                const double* src =
                    face_flux + ((((size_t)fine * 3 + d) * 2 + fside) * CELLS / SUB +
                                 face_index(fu & 7, fv & 7)) * nf;
                for (int f = 0; f < nf; ++f) Hf[i][j][f] = src[f];
              }
            const double* hc =
                face_flux + ((((size_t)c * 3 + d) * 2 + side) * CELLS / SUB + face_index(u, v)) * nf;
            int32_t l[3];
            l[d] = side ? SUB - 1 : 0;
            l[d == 0 ? 1 : 0] = u;
            l[d == 2 ? 1 : 2] = v;
            const int32_t cell = l[2] * 64 + l[1] * 8 + l[0];
            for (int f = 0; f < nf; ++f) {
              const double havg =
                  0.25 * ((Hf[0][0][f] + Hf[1][0][f]) + (Hf[0][1][f] + Hf[1][1][f]));
              const double q = (havg - hc[f]) * inv_dx;
              double* out = &Uout[((size_t)f * g->n_leaves + c) * CELLS + cell];
              *out = side ? *out - wdt * q : *out + wdt * q;
            }
          }
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Global time-step size (CFL condition on cell-centred signal speeds).     */
/* ------------------------------------------------------------------------ */

double oracle_cfl_dt(const ogrid* g, const double* U, double cfl) {
  double best = INFINITY;
#pragma omp parallel for reduction(min : best) schedule(static)
  for (int32_t n = 0; n < g->n_leaves; ++n) {
    const int32_t L = g->coord[4 * n + 0];
    const double dx = 1.0 / (double)(SUB * (g->base << L));
    for (int32_t cell = 0; cell < CELLS; ++cell) {
      double u[6];
      for (int f = 0; f < 6; ++f) u[f] = U[((size_t)f * g->n_leaves + n) * CELLS + cell];
      double rinv, p, c;
      eos(u, g->gamma, g->eta1, &rinv, &p, &c);
      const double vmax = fmax(fmax(fabs(u[1] * rinv), fabs(u[2] * rinv)), fabs(u[3] * rinv));
      const double q = dx / (vmax + c);
      if (q < best) best = q;
    }
  }
  return cfl * best;
}

/* ------------------------------------------------------------------------ */
/* Conserved totals: sum of q * dV over all cells, Neumaier-compensated.    */
/* ------------------------------------------------------------------------ */

void oracle_totals(const ogrid* g, const double* U, double* out) {
  for (int f = 0; f < g->nf; ++f) {
    double s = 0.0, comp = 0.0;
    for (int32_t n = 0; n < g->n_leaves; ++n) {
      const int32_t L = g->coord[4 * n + 0];
      const double dx = 1.0 / (double)(SUB * (g->base << L));
      const double dv = dx * dx * dx;
      for (int32_t cell = 0; cell < CELLS; ++cell) {
        const double x = U[((size_t)f * g->n_leaves + n) * CELLS + cell] * dv;
        const double t = s + x;
        if (fabs(s) >= fabs(x))
          comp += (s - t) + x;
        else
          comp += (x - t) + s;
        s = t;
      }
    }
    out[f] = s + comp;
  }
}

/* ------------------------------------------------------------------------ */
/* SSP-RK3 time step (Shu & Osher 1988): three substeps, Sec. I.            */
/* ------------------------------------------------------------------------ */

int64_t oracle_rk3_step(const ogrid* g, double* U, double* W1, double* W2, double cfl,
                        double dt_in, double* dt_out) {
  return oracle_rk3_step_reflux(g, U, W1, W2, cfl, dt_in, dt_out, 0);
}

int64_t oracle_rk3_step_reflux(const ogrid* g, double* U, double* W1, double* W2, double cfl,
                               double dt_in, double* dt_out, int reflux) {
  const double dt = dt_in > 0.0 ? dt_in : oracle_cfl_dt(g, U, cfl);
  const size_t total = (size_t)g->nf * g->n_leaves * CELLS;
  double* ff = reflux ? (double*)malloc(sizeof(double) * (size_t)g->n_leaves * 6 * 64 * g->nf)
                      : NULL;
  int64_t bad = 0;
  bad += oracle_step_record(g, NULL, U, W1, dt, 1.0, NULL, 0, ff);
  if (ff) oracle_reflux(g, W1, dt, 1.0, ff, NULL, 0);
  bad += oracle_step_record(g, U, W1, W2, dt, 0.25, NULL, 0, ff);
  if (ff) oracle_reflux(g, W2, dt, 0.25, ff, NULL, 0);
  bad += oracle_step_record(g, U, W2, W1, dt, 2.0 / 3.0, NULL, 0, ff);
  if (ff) oracle_reflux(g, W1, dt, 2.0 / 3.0, ff, NULL, 0);
  free(ff);
  memcpy(U, W1, sizeof(double) * total);
  if (dt_out) *dt_out = dt;
  return bad;
}

/* ------------------------------------------------------------------------ */
/* 1D periodic solver with the same reconstruction and flux (for pins).     */
/* ------------------------------------------------------------------------ */

/* q[nf][n] periodic along x with cell width 1/n; transverse momenta are
 * carried as fields 2 and 3.  One Runge-Kutta substep. */
int64_t oracle_step_1d(int32_t n, int nf, const double* U0, const double* Uk, double* Uout,
                       double dt, double beta, double gamma, double eta1) {
  const int32_t m = n + 2 * GH;
  double* ext = (double*)malloc(sizeof(double) * (size_t)nf * m);
  double* qL = (double*)malloc(sizeof(double) * (size_t)nf * m);
  double* qR = (double*)malloc(sizeof(double) * (size_t)nf * m);
  double* H = (double*)malloc(sizeof(double) * (size_t)nf * m);
  int64_t bad = 0;
  for (int f = 0; f < nf; ++f)
    for (int32_t k = 0; k < m; ++k) ext[(size_t)f * m + k] = Uk[(size_t)f * n + wrapi(k - GH, n)];
  /* PPM on overlapping windows of 14 so that every window sees the same
   * arithmetic as a 3D pencil. */
  for (int f = 0; f < nf; ++f)
    for (int32_t s = 0; s < n; s += SUB) {
      double win[TW], wl[TW], wr[TW];
      for (int k = 0; k < TW; ++k) win[k] = ext[(size_t)f * m + s + k];
      oracle_ppm_1d(win, TW, wl, wr);
      for (int k = GH - 1; k <= GH + SUB; ++k) {
        qL[(size_t)f * m + s + k] = wl[k];
        qR[(size_t)f * m + s + k] = wr[k];
      }
    }
  double UL[ORACLE_MAX_NF], UR[ORACLE_MAX_NF], h[ORACLE_MAX_NF];
  for (int32_t k = GH - 1; k < GH + n; ++k) {
    for (int f = 0; f < nf; ++f) {
      UL[f] = qR[(size_t)f * m + k];
      UR[f] = qL[(size_t)f * m + k + 1];
    }
    bad += oracle_face_flux(0, nf, UL, UR, gamma, eta1, h);
    for (int f = 0; f < nf; ++f) H[(size_t)f * m + k] = h[f];
  }
  const double inv_dx = (double)n;
  for (int f = 0; f < nf; ++f)
    for (int32_t i = 0; i < n; ++i) {
      const double d = H[(size_t)f * m + i + GH] - H[(size_t)f * m + i + GH - 1];
      const double zero = 0.0;
      const double lrate = -((d + zero) + zero) * inv_dx;
      combine(U0 != NULL, beta, dt, U0 ? U0[(size_t)f * n + i] : 0.0, Uk[(size_t)f * n + i], lrate,
              &Uout[(size_t)f * n + i]);
    }
  free(ext);
  free(qL);
  free(qR);
  free(H);
  return bad;
}

/* Threads an OpenMP parallel region of the oracle uses. */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Sets the threads of the oracle's later parallel regions (timing only). */
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
