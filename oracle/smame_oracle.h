/*
 * Plain FP64 CPU oracle for the SMAME step (Huang, "Towards the simplest
 * simulation of incompressible viscous flows inspired by the lattice
 * Boltzmann method", arXiv 2012.03525).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header or constant with the HIP library.
 *
 * Layout: every field is a dense FP64 array, x fastest, index
 * (k*ny + j)*nx + i (k = 0 in 2D).  Density is carried as the deviation
 * drho = rho - rho0.
 */
#ifndef SMAME_ORACLE_H
#define SMAME_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* face order: -x, +x, -y, +y, -z, +z */
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_SYMMETRY = 2 };

typedef struct {
    int dim, nx, ny, nz;        /* nz ignored (taken as 1) in 2D            */
    double dx, dt, nu, cs, rho0;
    double sat_rho, sat_mom;    /* multipliers of the two stabilising terms  */
    double g[3];                /* uniform body force                        */
    int bc[6];
    double wall_u[6][3];        /* wall velocity of each face                */
    int two_phase;              /* 2D or 3D                                  */
    double sigma, width, mobility;
    double wet_cos[6];          /* cos(contact angle) of each wall face;
                                   0 = 90 degrees (phi mirrored)             */
    int axisym;                 /* 2D: x is the axial coordinate, y the
                                   radius; the -y face is the axis (symmetry
                                   plane), node j at r = (j+1/2) dx          */
} orc_params;

/* One time step.  in_* are level n, out_* receive level n+1 (must not alias
 * the inputs).  w/phi (and out_w/out_phi) may be NULL when unused.
 * force_x_row: NULL or ny values added to g[0] on row j.
 * Returns 0 on success, -1 on invalid parameters, -2 on allocation failure. */
int orc_step(const orc_params* p, const double* force_x_row,
             const double* drho, const double* u, const double* v,
             const double* w, const double* phi,
             double* out_drho, double* out_u, double* out_v,
             double* out_w, double* out_phi);

/* nsteps steps, ping-ponging internally; the result is written back into
 * the in/out arrays. */
int orc_run(const orc_params* p, const double* force_x_row, long nsteps,
            double* drho, double* u, double* v, double* w, double* phi);

/* Diagnostics of one state (prev_* may be NULL: then out[5] = 0).
 * out[0]  mass      sum(drho) dx^D
 * out[1..3] momentum sum(rho u_a) dx^D
 * out[4]  E_k = 1/2 sum(|u|^2) dx^D
 * out[5]  max | |u| - |u_prev| |
 * out[6]  max |u|
 * out[7]  enstrophy (1/(2S)) sum |omega|^2 dS
 * out[8]  energy    (1/(2S)) sum |u|^2 dS
 * out[9]  rms of the centred divergence
 * out[10] max |centred divergence|
 * out[11] sum(phi)
 * out[12] 1 if any field value is not finite, else 0                     */
int orc_diag(const orc_params* p, const double* drho, const double* u,
             const double* v, const double* w, const double* phi,
             const double* prev_u, const double* prev_v, const double* prev_w,
             double* out);

/* Chemical potential mu = 4 a phi (phi^2-1) - kappa L_iso phi of a 2D or
 * 3D order-parameter field, with the ghost rules of the parameters. */
int orc_chemical_potential(const orc_params* p, const double* phi, double* mu);

#ifdef __cplusplus
}
#endif
#endif
