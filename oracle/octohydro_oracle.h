/*
 * octohydro_oracle.h -- interface of the FP64 CPU oracle (test infrastructure
 * only; see octohydro_oracle.c).  Independent of the library's public header.
 */
#ifndef OCTOHYDRO_ORACLE_H
#define OCTOHYDRO_ORACLE_H

#include <stdint.h>

#define ORACLE_MAX_NF 16

enum { ORACLE_SAME_LEAF = 0, ORACLE_SAME_REFINED = 1, ORACLE_COARSER_LEAF = 2 };
enum { ORACLE_OK = 0, ORACLE_E_ARG = -1, ORACLE_E_TABLE = -2 };

typedef struct {
  int32_t n_leaves, nf, base;
  const int32_t* coord;    /* [n_leaves][4]: level, ix, iy, iz */
  const int32_t* nbr;      /* [n_leaves][27] */
  const uint8_t* kind;     /* [n_leaves][27] */
  const int32_t* children; /* [n_nodes][8] */
  double gamma, eta1;
  double omega; /* frame angular velocity about the z axis through (0.5, 0.5) */
  int32_t recon; /* 0: PPM per axis, flux at the face centre;
                    1: 3D reconstruction, 9-point Simpson flux per face */
} ogrid;

int oracle_build_table(int32_t n_leaves, int32_t base, const int32_t* leaf_coord, int32_t* nbr,
                       uint8_t* kind, int32_t* children, int32_t max_nodes, int32_t* n_nodes_out);
void oracle_fill_ghosts(const ogrid* g, const double* U, double* G);
void oracle_ppm_1d(const double* q, int n, double* qL, double* qR);
int oracle_face_flux(int d, int nf, const double* UL, const double* UR, double gamma, double eta1,
                     double* H);
int64_t oracle_step(const ogrid* g, const double* U0, const double* Uk, double* Uout, double dt,
                    double beta);
/* Same substep, computed only for the leaves listed in subset (Uout of the
 * other leaves is left untouched). */
int64_t oracle_step_subset(const ogrid* g, const double* U0, const double* Uk, double* Uout,
                           double dt, double beta, const int32_t* subset, int32_t n_subset);
/* Same, also recording into face_flux (if not NULL) the fluxes through the
 * six faces of every processed leaf: [leaf][d][side][v][u][nf] with u, v the
 * other two axes in increasing order and side 0 = low face, 1 = high face. */
int64_t oracle_step_record(const ogrid* g, const double* U0, const double* Uk, double* Uout,
                           double dt, double beta, const int32_t* subset, int32_t n_subset,
                           double* face_flux);
void oracle_reflux(const ogrid* g, double* Uout, double dt, double w, const double* face_flux,
                   const int32_t* subset, int32_t n_subset);
int64_t oracle_rk3_step_reflux(const ogrid* g, double* U, double* W1, double* W2, double cfl,
                               double dt_in, double* dt_out, int reflux);
double oracle_cfl_dt(const ogrid* g, const double* U, double cfl);
void oracle_totals(const ogrid* g, const double* U, double* out);
int64_t oracle_rk3_step(const ogrid* g, double* U, double* W1, double* W2, double cfl,
                        double dt_in, double* dt_out);
int64_t oracle_step_1d(int32_t n, int nf, const double* U0, const double* Uk, double* Uout,
                       double dt, double beta, double gamma, double eta1);

/* 3D reconstruction (recon = 1): value of one field's 14^3 tile Tf at the
 * point t + p/2 of tile cell t (p in {-1,0,1}^3, not 0), and the 9-point
 * Simpson flux of the face normal to d between tile cells tl and tl + d
 * (T = nf consecutive tiles). */
double oracle_point_value(const double* Tf, const int32_t t[3], const int32_t p[3]);
int oracle_face_flux_3d(const ogrid* g, const double* T, int d, const int32_t tl[3], double* H);

int oracle_num_threads(void);
void oracle_set_num_threads(int n);

#endif
