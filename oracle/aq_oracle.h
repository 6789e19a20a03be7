/* Oracle of the coupled lattice Boltzmann model: types and entry points.
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing). */
#ifndef AQ_ORACLE_H
#define AQ_ORACLE_H
#include <stdint.h>

enum { OR_SOLID = 0, OR_FLUID = 1, OR_POROUS = 2, OR_INLET = 3, OR_OUTLET = 4 };
enum { OR_WALL_BOX = 0, OR_WALL_CORNEA = 1, OR_WALL_IRIS = 2 };

/* outlet_mode: 0 = pressure outlet at p_out; 1 = lumped trabecular meshwork (Darcy
 * seepage velocity from the IOP, applied as a velocity boundary condition) */
enum { OR_OUTLET_PRESSURE = 0, OR_OUTLET_LUMPED = 1 };
/* bc_scheme: 0 = half-way bounce-back walls; 1 = the paper's (section 2.3) interpolated
 * bounce-back of Bouzidi et al. on CORNEA and IRIS walls, with the wall list's fractions */
enum { OR_BC_LINKWISE = 0, OR_BC_PAPER = 1 };

typedef struct {
    int32_t nx, ny, periodic_x, periodic_y, check_interval, outlet_mode, bc_scheme, pad_;
    double tau_f, tau_t, w0;
    double u_in_x, u_in_y;
    double p_ref, p_out, p_init;
    double T_ref, T_init, T0;
    double T_cornea, T_iris, T_inlet;
    double gbeta, gravity_angle, K;
    double K_tm, h_tm, p_sc;   /* lumped meshwork: permeability, thickness, Schlemm's-canal pressure */
} or_params;

typedef struct {
    int64_t step;
    double iop_gauge, p_mean_fluid, q_in, q_out;
    double wss_cornea_mean, wss_cornea_max, wss_iris_mean, wss_iris_max;
    double resid_u, resid_T, u_max, mass_flow, mass_thermal;
    int64_t n_nonfinite;
    double u_seep;             /* lumped meshwork: seepage velocity for the next interval */
} or_observables;

typedef struct or_state or_state;

/* wall_q: [n_walls][8] link fractions (q[i-1] for link i; -1 where the link meets no wall) */
or_state* or_create(const or_params* P, const uint8_t* mask, int n_walls, const int32_t* wall_node,
                    const int32_t* wall_id, const double* wall_nx, const double* wall_ny, const double* wall_q);
void or_destroy(or_state* s);
void or_step(or_state* s, int64_t nsteps);
int64_t or_step_count(const or_state* s);
void or_set_outlet(or_state* s, double K_tm, double h_tm, double p_sc);
void or_observables_get(const or_state* s, or_observables* out);
/* The check-step observables of the current state, computed now (as a check step does,
 * including its update of the residual reference and of the lumped seepage speed). */
void or_observe(or_state* s, or_observables* out);
void or_fields(const or_state* s, double* dp, double* ux, double* uy, double* T);
void or_get_populations(const or_state* s, double* h, double* g);
void or_set_populations(or_state* s, const double* h, const double* g);
void or_collide_node(const or_params* P, int porous, const double* h8, const double* g5,
                     double* h8s, double* g5s);
void or_equilibrium(const or_params* P, double p, double ux, double uy, double T, double* h8, double* g5);
void or_moments(const or_params* P, const double* h8, const double* g5, double* out4);
void or_set_threads(int n);
int or_max_threads(void);
#endif
