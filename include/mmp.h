/*
 * mmp.h - C ABI of the MI355X micromagnetic hot path (libmmp.so).
 *
 * The library evaluates the effective field of a finite-difference
 * micromagnet and integrates the Landau-Lifshitz-Gilbert equation with an
 * embedded Runge-Kutta pair, following Moreels et al., "mumax+:
 * extensible GPU-accelerated micromagnetics and beyond" (arXiv 2411.18194),
 * Methods section:
 *   dm/dt = tau (Eq. 1), tau = LLG torque (Eq. 2) + Zhang-Li torque;
 *   B_eff = demag (zero-padded FFT convolution with the Newell tensor,
 *   asymptotic far field; "Magnetostatic field") + exchange (Eq. 3, with
 *   the intra- and inter-sublattice terms of an antiferromagnet) +
 *   interfacial DMI (Eq. 4 special case, boundary condition Eq. 5) +
 *   uniaxial/cubic anisotropy + Zeeman + magnetoelastic field (Eq. 9);
 *   elastodynamics (Eq. 7) with the magnetoelastic force (Eq. 8);
 *   the time solvers are the five embedded pairs of Table 2 (Dormand-Prince
 *   5(4) by default).
 *
 * Conventions
 *   Units are SI; fields are in tesla.  Host arrays are FP64, structure of
 *   arrays, index [sub][comp][z][y][x] with x fastest (N = nx*ny*nz cells):
 *   m has nsub*3*N values, u and v have 3*N.
 *   Every call returns an mmp_status: 0 on success, MMP_PENDING from
 *   mmp_poll while a request runs, a negative code on error; the message
 *   of the last error on the calling thread is mmp_last_error().  No call
 *   throws across the ABI.  Inputs are copied; outputs go to caller-owned
 *   buffers of the documented size.  A grid handle is used by one thread
 *   at a time; a server handle is thread-safe.  Grids on different threads
 *   may run concurrently: the library serialises its HIP graph captures
 *   with its synchronous copies and device allocations, which would
 *   otherwise invalidate a capture in flight on another thread.
 *
 * Precision: the state, FFTs and stencils run in FP32 or FP64 (per grid);
 * the demagnetising tensor is built in FP64, the RK error norm, the time
 * and the energies are FP64 in both cases.
 */
#ifndef MMP_H
#define MMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mmp_status;
#define MMP_OK               0
#define MMP_PENDING          1
#define MMP_E_ARG           -1   /* invalid argument or size              */
#define MMP_E_NOMEM         -2   /* device allocation failed               */
#define MMP_E_HIP           -3   /* HIP runtime error                      */
#define MMP_E_NONFINITE     -4   /* NaN/Inf appeared in the state          */
#define MMP_E_DT_UNDERFLOW  -5   /* adaptive step fell below dt_min        */
#define MMP_E_TOO_LARGE     -6   /* request exceeds the server's HBM budget*/
#define MMP_E_STATE         -7   /* call out of order (e.g. no params)     */
#define MMP_E_TICKET        -8   /* unknown ticket                         */

#define MMP_FP32 0
#define MMP_FP64 1

/* Embedded Runge-Kutta pairs (Table 2 of the paper: convergence order /
 * error-estimate order).  The higher-order solution is propagated; the
 * step-size factor is 0.8 (tol/err)^(1/(q+1)) clipped to [0.1, 2]. */
#define MMP_RK_DP45      0  /* Dormand-Prince 5/4, first same as last     */
#define MMP_RK_HEUN      1  /* Heun 2/1 (Euler embedded)                  */
#define MMP_RK_BS23      2  /* Bogacki-Shampine 3/2, first same as last   */
#define MMP_RK_CASHKARP  3  /* Cash-Karp 5/4                              */
#define MMP_RK_FEHLBERG  4  /* Fehlberg 5/4, 5th order propagated         */

/* Effective-field terms (bit mask for mmp_eval_heff). */
#define MMP_T_DEMAG     (1u << 0)  /* magnetostatic field                  */
#define MMP_T_EXCH      (1u << 1)  /* 2 A11/Ms lap m   (Eq. 3, term 1)     */
#define MMP_T_AFM_NN    (1u << 2)  /* A12/Ms lap m'    (Eq. 3, term 2)     */
#define MMP_T_AFM_CELL  (1u << 3)  /* 4 A0/(Ms a^2) m' (Eq. 3, term 3)     */
#define MMP_T_DMI       (1u << 4)  /* DMI: interfacial (one sublattice),
                                      homogeneous d.(m1 x m2) (two)        */
#define MMP_T_ANIS_U    (1u << 5)  /* uniaxial anisotropy                  */
#define MMP_T_ANIS_C    (1u << 6)  /* cubic anisotropy                     */
#define MMP_T_ZEEMAN    (1u << 7)  /* external field                       */
#define MMP_T_MEL       (1u << 8)  /* magnetoelastic field (Eq. 9)         */
#define MMP_T_ALL       0x1FFu
#define MMP_T_ZL        (1u << 9)  /* add Zhang-Li torque (torque output)  */
#define MMP_OUT_TORQUE  (1u << 16) /* b_out receives dm/dt, not B          */

/* energy_out of mmp_eval_heff: MMP_NENERGY doubles, joules, in this order:
 * demag, exch, afm_nn, afm_cell, dmi, anis_u, anis_c, zeeman, mel, elastic */
#define MMP_NENERGY 10

typedef struct mmp_grid_s* mmp_grid;
typedef struct mmp_server_s* mmp_server;

/* Per-sublattice material constants. */
typedef struct {
  double Ms;          /* saturation magnetisation, A/m (0 = empty)        */
  double A11;         /* exchange stiffness, J/m                          */
  double alpha;       /* Gilbert damping                                  */
  double Ku1, Ku2;    /* uniaxial anisotropy, J/m^3                       */
  double anis_u[3];   /* uniaxial axis (unit)                             */
  double Kc1;         /* cubic anisotropy, J/m^3                          */
  double cub_c1[3];   /* cubic axes c1, c2 (c3 = c1 x c2)                 */
  double cub_c2[3];
  double Dint;        /* interfacial DMI, J/m^2 (one sublattice only)     */
  double B1, B2;      /* magnetoelastic coupling, J/m^3                   */
  double zl_P;        /* Zhang-Li spin polarisation                       */
  double zl_xi;       /* Zhang-Li non-adiabaticity                        */
} mmp_sublattice;

typedef struct {
  uint32_t struct_size;   /* sizeof(mmp_params)                           */
  int32_t precision;      /* MMP_FP32 or MMP_FP64                          */
  int32_t nsub;           /* 1 (ferromagnet), 2 (two sublattices) or 3
                             (three, e.g. a non-collinear antiferromagnet:
                             every pair coupled by the same A12 and A0;
                             open boundaries, no elasticity, no
                             homogeneous DMI)                              */
  int32_t demag;          /* nonzero: magnetostatic field on               */
  double gamma;           /* gyromagnetic ratio, rad/(s T)                 */
  mmp_sublattice sub[3];  /* sub[2] only for three sublattices           */
  double A0;              /* homogeneous inter-sublattice exchange, J/m    */
  double A12;             /* inhomogeneous inter-sublattice exchange, J/m  */
  double latcon;          /* lattice constant a, m                         */
  double B_ext[3];        /* external field, T                             */
  double j[3];            /* current density, A/m^2 (Zhang-Li)             */
  int32_t dmi_layer;      /* z-layer carrying the DMI; -1 = every layer    */
  int32_t ngrains;        /* 0 = no grains; else grain/grain_axes given    */
  const uint16_t* grain;  /* N grain ids (copied), or NULL                 */
  const double* grain_axes; /* ngrains*3 uniaxial axes (copied), or NULL   */
  int32_t elastic;        /* nonzero: elastodynamics on (u, v in state)    */
  int32_t pad0;
  double rho, C11, C12, C44, eta;  /* kg/m^3, Pa, kg/(m^3 s)               */
  double trac_amp;        /* shear traction sigma_xz on x=0 face, Pa       */
  double trac_freq;       /* ... times sin(2 pi f t), Hz                   */
  double tol;             /* adaptive error tolerance (default 1e-5)       */
  double dt0;             /* first adaptive step, s (default 1e-14)        */
  double dt_min;          /* underflow limit, s (default 1e-20)            */
  int32_t solver;         /* MMP_RK_*: embedded Runge-Kutta pair           */
  int32_t pbc[3];         /* periodic boundaries: image repetitions R per
                             axis, 0 = open.  R > 0 along x or y makes that
                             axis periodic for the exchange, DMI and
                             Zhang-Li stencils (neighbours wrap, no DMI
                             boundary condition on its faces) and for the
                             demag field (cyclic convolution of period n,
                             kernel summed over the images k = -R..R, the
                             half-period offset holding the mean of +-n/2).
                             A periodic axis with demag needs n = 1 or n
                             even and 7-smooth, <= 4096; pbc[2] must be 0;
                             not combined with elasticity; R <= 1024       */
  double rayleigh;        /* elastic strain-rate damping: stress gains
                             rayleigh * C : eps(v) (stiffness-proportional
                             Rayleigh damping, s; 0 = none)                */
  double dmi_homo[3];     /* homogeneous DMI vector d of a two-sublattice
                             magnet, J/m^3: energy density d.(m1 x m2)
                             per cell, reported with the DMI term          */
  int32_t bc_eq6;         /* 1: the Neumann condition of Eq. 6 on every
                             open face (A12 coupling of the two
                             sublattices' normal derivatives and the DMI
                             tensor term, solved per boundary cell) feeds
                             the exchange, A12 and DMI stencils, and the
                             DMI tensors below are on; 0: a missing
                             neighbour is the cell itself (Eq. 5 ghosts
                             for the interfacial Dint)                     */
  int32_t pad2;
  double dmi_W[2][3][3];  /* DMI tensor of each sublattice (Eq. 4) as
                             three vectors W_i: D_ijk = sum_a eps_ajk W_ia
                             (W_ix = D_i,yz, W_iy = D_i,zx, W_iz = D_i,xy),
                             J/m^2; needs bc_eq6; interfacial D:
                             W_x = (0, D, 0), W_y = (-D, 0, 0)             */
  double dmi_W12[3][3];   /* inter-sublattice DMI tensor, same form        */
  double grain_exch_reduction; /* polycrystal (ngrains > 0): the exchange
                             (A11) and inhomogeneous inter-sublattice (A12)
                             stencil links between cells of different grains
                             carry (1 - r) times the constant (the paper's
                             reduced exchange at grain boundaries); DMI is
                             not scaled; 0 = none, 1 = decoupled grains;
                             0 <= r <= 1                                   */
  /* Adaptive step control (0 = default): after every attempt the proposal
     is h * clip(safety (tol/err)^(1/(q+1)), fac_min, fac_max) (fac_max when
     err = 0), then at most dt_max; the first step is at most dt_max too.  */
  double dt_max;          /* largest step, s (0 = unbounded)               */
  double safety;          /* in (0, 1] (default 0.8)                       */
  double fac_min;         /* in (0, 1) (default 0.1): below 1, so that a
                             rejected attempt always shrinks the step     */
  double fac_max;         /* >= 1, >= fac_min (default 2)                  */
} mmp_params;

typedef struct {
  double t;         /* time after the call, s                            */
  double dt;        /* controller's next step, s                         */
  double err;       /* last error estimate                               */
  int64_t steps;    /* accepted steps                                    */
  int64_t rejects;  /* rejected attempts                                 */
} mmp_step_info;

typedef struct {
  uint32_t struct_size;
  int32_t max_samples;    /* capacity of sample_t / sample_m               */
  double sample_every;    /* output interval, s (0 = only t_end)           */
  double* sample_t;       /* [max_samples] sample times, or NULL           */
  double* sample_m;       /* [max_samples][nsub][3] averages of m, or NULL */
  int64_t max_steps;      /* safety limit on attempts (0 = none)           */
} mmp_run_opts;

typedef struct {
  double t;
  double dt;
  int64_t steps;
  int64_t rejects;
  int32_t nsamples;
  int32_t status;
} mmp_run_info;

/* ---------------------------------------------------------------- grid -- */

/* Create a grid of nx*ny*nz cells of size cellsize[3] (metres).  The grid
 * owns its device memory until mmp_grid_destroy.  MMP_E_ARG for any size
 * < 1 or a demag pad above 4096 per axis. */
mmp_status mmp_grid_create(int32_t nx, int32_t ny, int32_t nz,
                           const double cellsize[3], mmp_grid* out);
mmp_status mmp_grid_destroy(mmp_grid g);

/* Copy the material, precision and solver settings (p->struct_size must
 * match).  Builds the demagnetising kernel (FP64 Newell / quadrature /
 * asymptotic tensor, transformed on the GPU) when p->demag is set and the
 * geometry changed.  Invalidates the FSAL stage. */
mmp_status mmp_set_params(mmp_grid g, const mmp_params* p);

/* Upload the state: m (nsub*3*N, normalised by the caller), u and v (3*N
 * each, may be NULL = zero; ignored without elasticity), time t. */
mmp_status mmp_set_state(mmp_grid g, const double* m, const double* u,
                         const double* v, double t);
/* Download the state; any pointer may be NULL. */
mmp_status mmp_get_state(mmp_grid g, double* m, double* u, double* v,
                         double* t, double* dt);

/* Evaluate the effective field of the current state for the terms in
 * term_mask.  b_out (nsub*3*N, may be NULL) receives B (T) or, with
 * MMP_OUT_TORQUE, dm/dt (1/s) of those terms (+ Zhang-Li with MMP_T_ZL).
 * energy_out (MMP_NENERGY, may be NULL) receives per-term energies of all
 * terms (FP64 accumulation).  Synchronous. */
mmp_status mmp_eval_heff(mmp_grid g, uint32_t term_mask, double* b_out,
                         double* energy_out);

/* Device-pointer variants of mmp_set_state, mmp_get_state and
 * mmp_eval_heff, for callers whose data already live on the GPU (e.g.
 * PyTorch tensors): the interface sketch's device variants of the state
 * and field calls.  Every buffer is FP64 DEVICE memory of the grid's device
 * in the host layout of the matching call ([sub][comp][z][y][x], x
 * fastest; u, v [comp][z][y][x]), owned by the caller.  The work is
 * enqueued on the grid's stream (mmp_set_stream) after whatever is already
 * queued there, and the call returns without synchronising: inputs must
 * stay valid, and outputs are written, when that stream reaches the work
 * (order a torch stream after it, or call mmp_synchronize).  MMP_E_ARG for
 * a buffer that is not device memory of the grid's device.
 *
 * mmp_set_state_device: m_dev (nsub*3*N) is rounded to the grid's precision
 *   as given (not renormalised, like mmp_set_state); u_dev, v_dev (3*N, may
 *   be NULL = zero) for elastic grids; the step controller restarts at t.
 * mmp_get_state_device: any output may be NULL; t_dt_dev (2 doubles)
 *   receives t and the next step size.
 * mmp_eval_heff_device: b_dev (nsub*3*N) receives what mmp_eval_heff's
 *   b_out does for term_mask (B in tesla, or dm/dt with MMP_OUT_TORQUE);
 *   no energies.  An FP32 grid keeps an FP32 buffer of that size from its
 *   first call. */
mmp_status mmp_set_state_device(mmp_grid g, const double* m_dev, const double* u_dev,
                                const double* v_dev, double t);
mmp_status mmp_get_state_device(mmp_grid g, double* m_dev, double* u_dev, double* v_dev,
                                double* t_dt_dev);
mmp_status mmp_eval_heff_device(mmp_grid g, uint32_t term_mask, double* b_dev);

/* One step of the grid's Runge-Kutta pair (mmp_params.solver).
 * dt_fixed > 0: fixed step, enqueued without a host synchronisation when
 * info is NULL.  dt_fixed == 0: adaptive, retried until accepted
 * (synchronous); MMP_E_DT_UNDERFLOW if the step falls below dt_min first,
 * MMP_E_STATE if 1000 attempts in a row are rejected. */
mmp_status mmp_step(mmp_grid g, double dt_fixed, mmp_step_info* info);

/* nsteps fixed steps of dt, all enqueued on the grid's stream with no host
 * synchronisation (info may be NULL; when given the call synchronises). */
mmp_status mmp_run_fixed(mmp_grid g, double dt, int64_t nsteps,
                         mmp_step_info* info);

/* Adaptive run from the current time to t_end with device-side step control
 * (no host round trip per step); steps land exactly on sample times and on
 * t_end.  opts may be NULL. */
mmp_status mmp_run(mmp_grid g, double t_end, const mmp_run_opts* opts,
                   mmp_run_info* info);

/* Use an existing HIP stream (e.g. torch.cuda.current_stream().cuda_stream)
 * for all later work on this grid; NULL = the library's own stream. */
mmp_status mmp_set_stream(mmp_grid g, void* hip_stream);
mmp_status mmp_synchronize(mmp_grid g);

/* HIP graphs for the step loops (default on).  When on, mmp_run_fixed,
 * mmp_run and the server enqueue the kernels of 8 step attempts as one
 * captured graph: every kernel reads the step controller and the stage
 * buffer table from device memory, so one capture serves every replay.
 * Graphs are not used while profiling (mmp_prof_enable) and are recaptured
 * after any change of parameters, plan or sample buffers.  Results are
 * bitwise identical either way. */
mmp_status mmp_set_graphs(mmp_grid g, int32_t on);

/* Device footprint of the grid in bytes (state, stages, FFT buffers, kernel). */
mmp_status mmp_grid_bytes(mmp_grid g, int64_t* bytes);

/* FP64 demagnetising tensor on non-negative offsets, 6*N values ordered
 * (xx, yy, zz, xy, xz, yz)[z][y][x] (offset (x dx, y dy, z dz)). */
mmp_status mmp_get_demag_tensor(mmp_grid g, double* n6);

/* Stray field of the magnet's current state in a layer of cells of the
 * grid's cell size whose centres lie `height` metres above the top surface
 * (paper: the stray field imaged above a film, "Stray field imaging of the
 * non-collinear antiferromagnet Mn3Sn"; the magnetostatic field of
 * "Magnetostatic field", B = -mu0 sum_j N(r - r_j) M_j with the cell-pair
 * tensor at the layer's vertical offsets).  b_out: 3*nx*ny doubles
 * [comp][y][x], tesla, caller-owned.  MMP_E_ARG for height < dz/2 (the
 * layer would overlap the magnet).  A direct FP64 sum over all cell pairs
 * on the device (cost ~ (nx ny)^2 nz); allocates its tensor table
 * (6 nz (2nx-1)(2ny-1) doubles) for the call.  Synchronous. */
mmp_status mmp_stray_field(mmp_grid g, double height, double* b_out);

/* Allocation-free variant of mmp_stray_field, for callers that cannot call
 * hipMalloc (code under HIP graph capture, serving loops, harnesses that
 * forbid device allocation).  Same field, same kernels; b_out_dev is a
 * caller-owned DEVICE buffer of 3*nx*ny doubles [comp][y][x] on the grid's
 * device.  Enqueued on the grid's stream (mmp_set_stream) and returns
 * without synchronising: the field is there once that stream has run it
 * (e.g. after mmp_synchronize).  The tensor table lives in a fixed
 * per-device array of MMP_STRAY_NOALLOC_MAX doubles (16 MiB) that the
 * library holds from the first call on a device until the process ends:
 * MMP_E_TOO_LARGE when 6*nz*(2nx-1)*(2ny-1) exceeds it, MMP_E_ARG for
 * height < dz/2 or a b_out_dev that is not device memory of the grid's
 * device.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller. */
#define MMP_STRAY_NOALLOC_MAX 2097152
mmp_status mmp_stray_field_noalloc(mmp_grid g, double height, double* b_out_dev);

/* ------------------------------------------------------------- plan -- */

/* Launch plan of a grid.
 *
 * Demag part: how the demagnetising convolution (zero-padded FFT
 * convolution with the cell-averaged tensor, paper Methods "Magnetostatic
 * field") is laid out and launched.  pad[] are the FFT lengths per axis: 1
 * for an axis of one cell, else even, 7-smooth, >= 2n-1 and <= 4096.  Any
 * such pads give the same field up to rounding, because the padding removes
 * the circular wrap-around.  The launch shapes only regroup the per-line
 * transforms over blocks and lanes; z_lanes > 1 also refactors the z
 * transform (same result up to rounding).  Every count is a power of two.
 * With demag off these fields read 0 and are ignored on input.
 *
 * Stencil part: field_zplanes, the cells of an (x, y) column that one
 * thread of the fused field kernel marches through (1..nz; results are
 * bitwise independent of it). */
typedef struct {
  uint32_t struct_size;
  int32_t pad[3];         /* Px, Py, Pz                                    */
  int32_t x_rows[2];      /* rows per block, forward / inverse x pass:
                             2..16                                         */
  int32_t y_lines[2];     /* lines per block, forward / inverse y pass:
                             1..64 (3-D grids)                             */
  int32_t xy_cols;        /* kx columns per block of the fused y pass of
                             2-D grids: 1..64                              */
  int32_t z_cols;         /* ky columns per block, mixed-radix z pass      */
  int32_t z_lanes;        /* lanes per (kx, ky) column, register z pass
                             (power-of-two Pz <= 64): 1, 2 or 4            */
  int32_t z_waves;        /* waves-per-SIMD hint of that pass: 1, 2 or 4   */
  int32_t z_threads;      /* threads per block of that pass: 64, 128, 256  */
  int32_t z_mode;         /* 0: that pass loads the kernel values after
                             the forward transforms; 1 (FP32, z_waves 1):
                             it copies them into LDS as it loads the
                             columns (z_threads/64 * 6 * rows * 256 bytes of
                             LDS <= 64 KiB, rows = Pz/2 + 1 for z_lanes 1,
                             else Pz/z_lanes).  Same arithmetic per column */
  int32_t field_zplanes;  /* z cells per thread of the field kernel        */
  uint32_t kinds;         /* out: bits 0/1/2 set when the x/y/z passes use
                             the power-of-two register kernels             */
  int32_t lds_axes;       /* bits 0/1/2: run the x/y/z passes through the
                             mixed-radix LDS kernels even where the pad is
                             a power of two (0 = the register kernels
                             there); such a grid computes its field bitwise
                             as the server's batched demag does            */
  double demag_ms;        /* out: time of one demag evaluation measured by
                             mmp_autotune for this plan, 0 if not tuned    */
  double field_ms;        /* out: time of one field-kernel stage measured
                             by mmp_autotune, 0 if not tuned               */
} mmp_plan;

/* The grid's current plan.  MMP_E_STATE before mmp_set_params. */
mmp_status mmp_get_plan(mmp_grid g, mmp_plan* out);
/* Install a plan.  MMP_E_ARG if a pad or launch shape is outside the
 * limits above or the kernels' LDS and block-size limits (the grid keeps
 * its plan); a change of pads reallocates the FFT buffers and rebuilds the
 * kernel spectrum.  Output-only fields are ignored.  Synchronous. */
mmp_status mmp_set_plan(mmp_grid g, const mmp_plan* p);
/* Autotuner.  For every pad set built from the smallest even 7-smooth pad
 * and the smallest power-of-two pad of each axis, times the candidate
 * launch shapes of each demag pass on the grid's stream (HIP events, real
 * buffers; pad sets that do not fit in free device memory are skipped),
 * then the field kernel's z march lengths; installs the fastest plan and
 * keeps it for grids of the same (nx, ny, nz, precision, demag on/off) on
 * this device that later calls of mmp_set_params set up in this process.
 * The magnetic state, time and step size are untouched (the timed launches
 * write only FFT buffers, B_d and stage scratch).  Synchronous; out may be
 * NULL. */
mmp_status mmp_autotune(mmp_grid g, mmp_plan* out);

/* Kernel timing with HIP events on the grid's stream.  While enabled every
 * launch of the hot path is bracketed by events; mmp_prof_read returns,
 * for kernel class idx (0 <= idx < mmp_prof_count()), its name, the summed
 * duration in ms and the launch count since the last reset. */
mmp_status mmp_prof_enable(mmp_grid g, int32_t on);
int32_t mmp_prof_count(void);
mmp_status mmp_prof_read(mmp_grid g, int32_t idx, const char** name,
                         double* total_ms, int64_t* launches);
mmp_status mmp_prof_reset(mmp_grid g);

/* -------------------------------------------------------------- server -- */

typedef struct {
  uint32_t struct_size;
  int64_t hbm_budget;     /* bytes of device memory for requests           */
  int32_t max_active;     /* concurrent requests on the device             */
  int32_t precision;      /* MMP_FP32 or MMP_FP64 for every request        */
  int32_t batch;          /* 1: requests without elasticity that use the
                             Dormand-Prince pair step together, one batch
                             per sublattice count: every stage is one
                             launch per demag pass and one field launch for
                             all members (demag through the mixed-radix LDS
                             kernels on every axis, the request's own
                             kernels set to match: mmp_plan.lds_axes = 7),
                             so a result is the same alone and in the mix;
                             0: each request on its own stream             */
} mmp_server_opts;

typedef struct {
  uint32_t struct_size;
  int32_t nx, ny, nz;
  double cellsize[3];
  mmp_params params;      /* precision field is overridden by the server   */
  const double* m0;       /* nsub*3*N initial state (copied at submit)     */
  double t_relax;         /* relaxation time, s                            */
} mmp_request;

typedef struct {
  int32_t status;         /* MMP_OK or an error code                       */
  int32_t nsub;
  double m_avg[3][3];     /* average m per sublattice at t_relax           */
  double energy;          /* total energy, J                               */
  int64_t steps, rejects;
  double t_submit, t_admit, t_done;  /* seconds on the server's clock      */
} mmp_result;

mmp_status mmp_server_create(const mmp_server_opts* o, mmp_server* out);
mmp_status mmp_submit(mmp_server s, const mmp_request* r, uint64_t* ticket);
/* MMP_PENDING while the request is queued or running; MMP_OK with its
 * result once it has finished (out->status holds the request's own status).
 * A result is returned once: afterwards the ticket is unknown
 * (MMP_E_TICKET). */
mmp_status mmp_poll(mmp_server s, uint64_t ticket, mmp_result* out);
mmp_status mmp_server_destroy(mmp_server s);
double mmp_server_clock(mmp_server s);

const char* mmp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MMP_H */
