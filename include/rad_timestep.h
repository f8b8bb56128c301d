/*
 * rad_timestep.h — time-dependent surface temperatures on one AMD Instinct
 * MI355X (gfx950): the time stepper of Potter et al., arXiv 2209.07632,
 * section 5.2 and Algorithm 6.
 *
 * Each step multiplies once by the compressed view-factor matrix per band
 * (reflected sunlight and thermal infrared; both bands go through one
 * product of 2R columns), so higher orders of scattering lag behind in time
 * as Algorithm 6 prescribes:
 *   Q_refl' = F diag(albedo) (Q_dir' + Q_refl)
 *   Q_IR'   = F (Q_rad + (1 - emiss) Q_IR)
 *   Q_abs'  = (1 - albedo) (Q_dir' + Q_refl') + emiss Q_IR'
 * and then advances a one-dimensional column of M layers under every facet by
 * one Crank-Nicolson step driven by Q_abs and Q_abs', which gives the new
 * surface temperature and Q_rad' = emiss sigma T_0'^4.
 *
 * Column scheme (section 5.2 leaves the discretisation to its reference):
 * nodes z_0 = 0 < z_1 < ... < z_M, a finite volume of half a layer on each
 * side of nodes 1..M (half a layer at the bottom, which receives the fixed
 * flux H); conduction is averaged over the two time levels (Crank-Nicolson).
 * The surface node has one of two readings (rad_ts_params.surface):
 *  - RAD_TS_SURFACE_HALF_LAYER: a volume of half a layer that receives
 *    Q_abs - emiss sigma T_0^4 (the radiation boundary condition of section 2),
 *    Q_abs averaged over the two levels and the emission averaged with its new
 *    value linearised about the old surface temperature.  Accurate for steps
 *    short against the top layer's diffusion time (on centimetre top layers
 *    about 0.3 K up to dt = 0.03 day, 2.8 K at 0.1 day, 24 K at 0.3 day);
 *  - RAD_TS_SURFACE_BALANCED: no heat capacity at the surface, which meets
 *    the radiation boundary condition at the new level,
 *    Q_abs' + k (T_1' - T_0') / z_1 = emiss sigma T_0'^4, solved by Newton's
 *    method on that one row (newton repeats after the first linearisation);
 *    accurate at the long steps of a lunation (0.5 K at 0.3 day on the same
 *    layers).
 * The M + 1 unknowns of a column form a tridiagonal system, eliminated from
 * the bottom up.
 *
 * R independent scenarios (for example R different sun sequences over the
 * same terrain) advance together.  Conventions as in rad.h: status codes,
 * rad_last_error(), caller-owned device pointers on the matrix's device, work
 * enqueued on hip_stream (NULL: the null stream) without waiting.  Calls on
 * one stepper, and calls on its matrix, must be serialised by the caller.
 *
 * Precision: column temperatures, Q_abs and Q_rad are kept in FP64; the
 * terrain fluxes are products by F-hat in the matrix's storage precision
 * (RAD_F64 or RAD_F32), and Q_dir inputs are in that precision (the layout
 * rad_insolation writes).  Everything rad_ts_read returns is FP64.
 */
#ifndef RAD_TIMESTEP_H
#define RAD_TIMESTEP_H

#include "rad.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rad_ts rad_ts;

typedef struct {
    int32_t n_layers;      /* M, 1 <= M <= 127                                           */
    const double *z;       /* host: M + 1 node depths (m), z[0] = 0, strictly increasing  */
    double conductivity;   /* k > 0 (W m^-1 K^-1)                                         */
    double heat_capacity;  /* volumetric heat capacity rho c > 0 (J m^-3 K^-1)            */
    double dt;             /* time step > 0 (s)                                           */
    double albedo;         /* in [0, 1)                                                   */
    double emissivity;     /* in (0, 1]                                                   */
    double bottom_flux;    /* H: heat flux entering every column from below (W m^-2)      */
    int32_t surface;       /* rad_ts_surface: reading of the surface node (default half layer) */
    int32_t newton;        /* balanced surface: Newton repeats after the first linearisation,
                              0 .. 16 (3 is enough for 1e-9 K at 0.3-day steps)          */
} rad_ts_params;

/* Reading of the surface node of every column (see the scheme above). */
typedef enum { RAD_TS_SURFACE_HALF_LAYER = 0, RAD_TS_SURFACE_BALANCED = 1 } rad_ts_surface;

/* Fields of the state, for rad_ts_read. */
typedef enum {
    RAD_TS_T = 0,      /* column temperatures: M + 1 blocks (node j = 0 is the surface) */
    RAD_TS_QABS = 1,   /* absorbed flux Q_abs of the current level                     */
    RAD_TS_QREFL = 2,  /* reflected short-wave flux Q_refl                             */
    RAD_TS_QIR = 3,    /* thermal infrared flux Q_IR                                   */
    RAD_TS_QRAD = 4    /* emitted flux Q_rad                                           */
} rad_ts_field;

/*
 * Creates a stepper for R scenarios on the single-instance matrix H (groups
 * are not supported: RAD_EUNSUP).  Needs 2 R <= max_rhs of H.  Copies p and
 * p->z; allocates the state on H's device: two sets of column temperatures
 * (2 (M+1) N R FP64 values), Q_abs and Q_rad (N R FP64 each) and the operand
 * and product of the 2R-column multiply.  The stepper must be freed before H.
 * Errors: RAD_EINVAL for a null pointer or a parameter outside the ranges
 * above (non-finite values included).
 */
rad_status rad_ts_create(const rad_hmat *H, const rad_ts_params *p, int64_t R, rad_ts **out);

/*
 * Level 0 of Algorithm 6: column temperatures from T0 (device, FP64, M + 1
 * blocks of N x R, block j at T0 + j * blk with blk = R * ldt in the
 * column-major orders and N * ldt in RAD_ORDER_TREE_RMAJOR); Q_abs = Q_rad =
 * (1 - albedo) Q_dir^(0) + H0 whatever T0 is, and Q_refl = Q_IR = 0, as the
 * algorithm initialises them.  Qdir0: device, N x R in the matrix's storage
 * precision.  order and the leading dimensions follow rad.h's rad_order
 * (RAD_ORDER_TREE_RMAJOR: ld equal to R rounded up to 4).
 */
rad_status rad_ts_init(rad_ts *S, const double *T0, int64_t ldt, const void *Qdir0, int64_t ldq, double H0,
                       int32_t order, void *hip_stream);

/*
 * Advances n_steps >= 1 levels.  Qdir: device, the direct insolation of the
 * levels n+1 .. n+n_steps (n = rad_ts_level), each an N x R block in the
 * matrix's storage precision, level i at Qdir + i * level_stride elements
 * (level_stride at least the block's extent).  Per step: one product by
 * F-hat of 2R columns and one kernel that forms Q_abs', steps every column,
 * and writes the next step's operand.  Errors: RAD_EINVAL before rad_ts_init
 * or for bad sizes.
 */
rad_status rad_ts_step(rad_ts *S, int64_t n_steps, const void *Qdir, int64_t ldq, int64_t level_stride,
                       int32_t order, void *hip_stream);

/*
 * Copies one field of the current level to out (device, FP64): an N x R
 * block, or M + 1 blocks for RAD_TS_T laid out as T0 of rad_ts_init.
 */
rad_status rad_ts_read(const rad_ts *S, int32_t field, double *out, int64_t ld, int32_t order, void *hip_stream);

/*
 * Diagnostic timing of the column kernel alone: nrep launches on the current
 * state (each advances every column from the current level into the spare
 * buffer, with the last product and operand standing in for the next level's
 * fluxes; the state's Q_abs and Q_rad are overwritten, so call rad_ts_init
 * again before using the stepper), timed with HIP events on hip_stream.
 * ms receives the average milliseconds per launch.
 */
rad_status rad_ts_time_column(rad_ts *S, int32_t nrep, void *hip_stream, double *ms);

/* Current level n (0 after rad_ts_init, -1 before); -1 for a null stepper. */
int64_t rad_ts_level(const rad_ts *S);

/* Frees the stepper (NULL is ignored). */
void rad_ts_free(rad_ts *S);

#ifdef __cplusplus
}
#endif

#endif /* RAD_TIMESTEP_H */
