/*
 * lb.h -- C ABI of the MI355X (gfx950) two-component colour-gradient lattice
 * Boltzmann library.
 *
 * The library advances two immiscible fluids A and B (total density
 * rho = rho_A + rho_B, phase field phi = (rho_A - rho_B)/rho) on a D2Q9, D3Q19
 * or D3Q27 lattice with pull streaming, BGK collision with body forcing, the
 * colour-gradient surface-tension perturbation, Latva-Kokko recolouring and
 * the near-contact repulsive force between approaching interfaces
 * (paper: Sec. III.B, Eqs. lbm and disteq; Sec. III.C.1, Eqs. CGLBE, ome3_1,
 * ome3_2, near_cont_force; Sec. III.D boundary conditions; Sec. IV "Second
 * group" for shifted storage).
 *
 * Conventions shared by every call:
 *  - Return value: LB_OK (0) or a negative lb_status.  No exception or C++
 *    type crosses the ABI.  lb_last_error() returns a thread-local message
 *    for the most recent failure on the calling thread.
 *  - Ownership: a handle owns all of its device memory (two population
 *    buffers, the phase field and the macroscopic field buffers).  The caller
 *    owns every buffer it passes in; the library never keeps a pointer to it
 *    after the call returns.
 *  - Streams: all device work of a handle is ordered on the HIP stream given
 *    to lb_create (NULL = the legacy default stream).  Calls with a host
 *    destination synchronise that stream before returning; calls with a
 *    device destination only enqueue.
 *  - Layout: sites are numbered s = x + nx*(y + ny*z), x fastest.  Populations
 *    are structure-of-arrays f[k][i][s] (k = 0 for A, 1 for B; i the velocity
 *    index).  The velocity numbering is the one lb_lattice_table reports; for
 *    D2Q9 it is the numbering the paper's boundary equations use.
 *  - Threading: a handle is not thread-safe.  Separate handles are independent.
 *  - One GPU: the handle lives on the device that is current when lb_create
 *    is called.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lb_status {
  LB_OK = 0,
  LB_EINVAL = -1,      /* invalid argument (bad size, enum, tau <= 1/2, channel, mask ...) */
  LB_ENOMEM = -2,      /* device allocation failed                                        */
  LB_EHIP = -3,        /* a HIP runtime call failed; lb_last_error() names it             */
  LB_ENUMERIC = -4,    /* watchdog: NaN/Inf, rho <= 0 or |u| > 0.3 found by a check       */
  LB_ENODEV = -5,      /* no HIP device                                                   */
  LB_EUNSUPPORTED = -6 /* valid request this build does not implement                     */
} lb_status;

typedef enum lb_lattice { LB_D2Q9 = 0, LB_D3Q19 = 1, LB_D3Q27 = 2 } lb_lattice;

/* Storage of the populations.  Collision arithmetic is FP64 for LB_F64 and
 * FP32 otherwise, in both cases on populations shifted by the rest
 * equilibrium (paper: Sec. IV "Second group", Eqs. shift_f, shift-lbm,
 * shift-eq).
 *  - Per-colour layouts keep both colours f^k_i.  LB_F64 / LB_F32 store f^k_i;
 *    LB_F32_SHIFTED and the 16-bit modes store the shifted
 *    f^k_i - w_i rho0 / 2 (Eq. shift_f per colour; 16-bit: rounded to
 *    nearest even).  LB_F16_SHIFTED and LB_BF16_SHIFTED are experimental:
 *    each step stores the correctly rounded values, but the per-colour split
 *    does not survive 16-bit rounding over many steps (velocity error of the
 *    order of the velocity itself after 200 steps of a 64^3 emulsion, against
 *    3e-3 for LB_F16_TOTAL); use the total layouts for 16-bit storage.
 *  - Total layouts keep the total post-collision population shifted by the
 *    rest equilibrium, T_i = f*_i - w_i rho0 (Eq. shift_f with rho0, u0 = 0), in
 *    the storage type, plus four FP32 scalars per site, a = rho_A / rho and
 *    b = beta (rho_A rho_B / rho) n (n the unit colour gradient).  The
 *    recolouring equations (Eqs. ome3_1, ome3_2) give the colours exactly:
 *    f^A_i = a f*_i + (w_i / |c_i|) c_i . b, f^B_i = f*_i - f^A_i.  The two-colour
 *    step is unchanged; the state is Q storage values + 16 bytes per site.
 *  - LB_F16C_TOTAL stores T_i in FP16C, the custom 16-bit format the paper
 *    cites for shifted populations (Sec. IV.A, second group): 1 sign, 4
 *    exponent (bias 15) and 11 significand bits, i.e. binary16 with one more
 *    significand bit and half its rounding error; normal magnitudes
 *    2^-14 .. 2 - 2^-11, subnormals in steps of 2^-25, no infinities (values
 *    beyond the largest saturate).  Rounded to nearest, ties to even. */
typedef enum lb_storage {
  LB_F64 = 0,
  LB_F32 = 1,
  LB_F16_SHIFTED = 2,
  LB_BF16_SHIFTED = 3,
  LB_F32_TOTAL = 4,
  LB_F16_TOTAL = 5,
  LB_BF16_TOTAL = 6,
  LB_F16C_TOTAL = 7,
  LB_F32_SHIFTED = 8
} lb_storage;

/* Near-contact force: off; the explicit scan (Eq. near_cont_force); or the
 * learned closure (3D lattices; storages LB_F64, LB_F32 and the total layouts)
 * with the explicit scan at interface sites outside the closure's input range. */
typedef enum lb_nc_mode { LB_NC_OFF = 0, LB_NC_EXPLICIT = 1, LB_NC_MLP = 2 } lb_nc_mode;

/* Streaming of the populations (paper Sec. IV.A, first group of memory
 * strategies).
 *  LB_STREAM_TWO_COPIES  each step pulls from one copy of the state into the
 *                        other.
 *  LB_STREAM_IN_PLACE    one copy, updated in place by the AA pattern: steps
 *                        alternate between a kind that pulls from the
 *                        neighbours and pushes back to them and a kind that
 *                        reads and writes only the site's own slots.  Halves
 *                        the memory of the populations (and of the total
 *                        layouts' recolouring scalars); same bytes per step,
 *                        same results bit for bit.  Single lattices only. */
typedef enum lb_streaming { LB_STREAM_TWO_COPIES = 0, LB_STREAM_IN_PLACE = 1 } lb_streaming;

/* What the state holds between steps (paper Sec. IV.A, third group of
 * memory strategies).
 *  LB_SCHEME_POPULATIONS  the post-collision populations (storage above).
 *  LB_SCHEME_MOMENTS      15 moments per site, from which the post-collision
 *      colours are rebuilt exactly; the step is the regularised one: the
 *      pulled total population enters BGK only through its projection on the
 *      second-order Hermite subspace (rho, j - rho u and
 *      Pi^neq = Pi - rho c_s^2 I - rho u u; Eqs. distnoneq, LBpostmom,
 *      llb-pull), then Guo source, perturbation and recolouring as usual.
 *      Moments, channel-major [15][N] in the storage type (LB_F64 or LB_F32):
 *        0 rho - rho0, 1-3 J = rho u + (1 - omega)(j - rho u) + (1 - omega/2) F,
 *        4-9 S (xx yy zz xy xz yz)
 *            = rho u u + (1 - omega) Pi^neq + (1 - omega/2)(u F + F u) + (2A/9) g g/|g|,
 *        10 s = A |g|, 11 a = rho_A / rho, 12-14 b = beta (rho_A rho_B / rho) g/|g|;
 *      P_i = w_i [rho + 3 c_i.J + 4.5 (c_i c_i - I/3) : S] + (2/3)(delta_i0 - w_i) s,
 *      P^A_i = a P_i + (w_i/|c_i|) c_i.b.  2D keeps the z channels at zero.
 *      Single lattices, two-copy streaming, nc_mode off or explicit. */
typedef enum lb_scheme { LB_SCHEME_POPULATIONS = 0, LB_SCHEME_MOMENTS = 1 } lb_scheme;

/* Rounding of the stored totals of LB_F16_TOTAL and LB_BF16_TOTAL (no other
 * storage takes a setting other than the default).
 *  LB_ROUND_NEAREST     nearest value, ties to even (the default).
 *  LB_ROUND_STOCHASTIC  one of the two neighbouring 16-bit values, the upper
 *                       one with probability equal to the value's fractional
 *                       position between them (the MI355X's stochastic
 *                       conversion), driven by a deterministic 32-bit word per
 *                       store: (h + i * 0x9E3779B9) exclusive-or the FP32
 *                       value's bits, with h = lowbias32 (C. Wellons' integer
 *                       hash) of site * 0x9E3779B9 + step * 0x85EBCA6B, one
 *                       hash per site and step.  Runs repeat bit for
 *                       bit, and in-place and two-copy streaming give the same
 *                       values.  Single lattices, nc_mode off or explicit. */
typedef enum lb_rounding { LB_ROUND_NEAREST = 0, LB_ROUND_STOCHASTIC = 1 } lb_rounding;

/* How a step forms the phase field its colour gradient needs, that of the
 * neighbours after streaming (Sec. III.C.1).  Both ways give the same step up
 * to the rounding order of the colour sums.
 *  LB_PHASE_SCATTER  read-once step: the collision pass of step t adds every
 *                    post-collision value, as storage will return it, to the
 *                    colour densities of the site that pulls it at step t+1
 *                    (x + c_i, or x itself when x + c_i is solid), so the
 *                    populations are read once per step; values that leave a
 *                    collision tile are summed into its halo block and a
 *                    small combine pass finishes the phase field.  The first
 *                    step after lb_init_droplets / lb_set_state first scatters
 *                    the stored state (a bootstrap pass that forms exactly the
 *                    sums the collision pass storing it formed), so restarts
 *                    repeat uninterrupted runs bit for bit.  Population
 *                    scheme, single lattices and ensembles (all channels
 *                    take the same phase_pass).
 *  LB_PHASE_PASS     a separate pass pulls the populations a second time each
 *                    step and forms the phase field before the collision pass
 *                    (the moment scheme always works this way).
 *  LB_PHASE_AUTO     (the default) the read-once step for the per-colour
 *                    layouts and LB_F32_TOTAL, the phase pass for the 16-bit
 *                    total layouts, whose collision pass is bound by
 *                    instruction issue and measured slower with the scatter. */
typedef enum lb_phase_mode { LB_PHASE_AUTO = 0, LB_PHASE_SCATTER = 1, LB_PHASE_PASS = 2 } lb_phase_mode;

/* field selection bits for lb_fields; dst[k] belongs to bit k */
enum {
  LB_FIELD_RHO_A = 1u << 0,   /* real[N]                                   */
  LB_FIELD_RHO_B = 1u << 1,   /* real[N]                                   */
  LB_FIELD_PHI = 1u << 2,     /* real[N]                                   */
  LB_FIELD_U = 1u << 3,       /* real[3][N]  (u_x block, u_y, u_z)         */
  LB_FIELD_FNC = 1u << 4,     /* real[3][N]  near-contact force density    */
  LB_FIELD_FLAGS = 1u << 5,   /* uint8[N]    1 where |phi| < phi_interface */
  LB_FIELD_LABELS = 1u << 6   /* int32[N]    droplet label or -1           */
};
#define LB_NUM_FIELDS 7

typedef struct lb_params {
  int lattice;            /* lb_lattice                                                  */
  int storage;            /* lb_storage                                                  */
  int nc_mode;            /* lb_nc_mode                                                  */
  int nx, ny, nz;         /* sites per axis; nz must be 1 for D2Q9                       */
  int wall[3];            /* per axis: 0 periodic, 1 halfway bounce-back wall on both faces */
  double tau;             /* BGK relaxation time of colour A (of both if tau_b == 0), > 1/2;
                             nu = (tau - 1/2)/3                                          */
  double A;               /* perturbation amplitude A = A_A = A_B                        */
  double beta;            /* recolouring parameter                                       */
  double rho0;            /* reference total density (initial state and storage shift)   */
  double body_force[3];   /* force density added at every site                           */
  double u0[3];           /* uniform velocity of the initial equilibrium                 */
  double nc_A;            /* near-contact plateau strength A_h for h <= nc_hmin          */
  double nc_hmin;         /* plateau end (sites); A_h = nc_A (nc_hmin/h)^3 beyond        */
  double nc_hmax;         /* scan range (sites), 1 <= nc_hmax <= 3                       */
  double phi_interface;   /* interface flag threshold phi_I in (0, 1)                    */
  int diag_every;         /* run the watchdog every this many steps inside lb_step (0 = never) */
  int streaming;          /* lb_streaming                                                */
  double tau_b;           /* relaxation time of colour B, > 1/2, or 0 for one viscosity.
                             Different viscosities mix per site (paper Sec. III.C.1, the
                             rule stated with the surface tension, Eq. sigmaA):
                             1/nu = (rho_A/rho)/nu_A + (rho_B/rho)/nu_B, and BGK and the
                             forcing use tau = 3 nu + 1/2                                */
  int scheme;             /* lb_scheme                                                   */
  int rounding;           /* lb_rounding                                                 */
  int phase_pass;         /* lb_phase_mode                                               */
} lb_params;

typedef struct lb_handle lb_handle;

/* Launch configuration of an ensemble step (n_channels > 1).
 *  mode          LB_ENSEMBLE_BATCHED: two launches per step over all channels
 *                (read-once step: every channel's collision tile-marches with
 *                the scatter, then every channel's combine blocks; two-pass
 *                step: every channel's phase tiles, then every channel's
 *                collision tiles; one tile per workgroup).
 *                LB_ENSEMBLE_PER_CHANNEL: the single-lattice launches of
 *                each channel's step, channel after channel; without the
 *                watchdog, lb_step(n) takes each channel through all n steps
 *                before the next channel (same results, bit for bit; the
 *                channel's state stays in the last-level cache).
 *  z_per_block   z-planes per collision tile (>= 1)
 *  use_graph     1: replay non-field steps from a captured hipGraph of two steps
 *                (batched mode; the per-channel mode launches directly and
 *                lb_autotune tries it without a graph only).  Single lattices
 *                (default 0) replay pairs of non-field steps at the buffer
 *                parities they were captured at; not with the watchdog, while
 *                profiling, before the read-once phase field is ready or with
 *                stochastic rounding (its key is the step count)
 *  ms_per_step   filled by lb_autotune with the measured time of the choice */
enum { LB_ENSEMBLE_BATCHED = 0, LB_ENSEMBLE_PER_CHANNEL = 1 };
typedef struct lb_tuning {
  int mode;
  int z_per_block;
  int use_graph;
  int reserved;           /* 0 */
  double ms_per_step;
} lb_tuning;

/* Fill *p with defaults: D3Q27, FP32, nc off, 64^3 periodic, tau 1, A 0.01,
 * beta 0.7, rho0 1, no force, u0 = 0, nc_A 0.02, hmin 2, hmax 3, phi_I 0.9. */
void lb_params_default(lb_params* p);

/* Create a simulation.  p points at n_channels parameter sets (1 .. 2048).
 * With n_channels > 1 the handle is an ensemble of independent lattices
 * ("channels") with their own sizes, walls, tau, forces and droplets, advanced
 * together by batched launches (lb_tuning); lattice, storage and nc_mode must
 * agree across channels and the storage must be LB_F64, LB_F32 or a total
 * layout, and nc_mode LB_NC_MLP is single-lattice only.  hip_stream is a
 * hipStream_t (NULL allowed).  Allocates two copies of the state (see
 * lb_state_bytes), or one with LB_STREAM_IN_PLACE, plus the fields, per
 * channel.  The population rows are kept padded to a multiple of 128 bytes on
 * the device (up to 63 16-bit, 31 FP32 or 15 FP64 extra sites per row; not in
 * the moment scheme); lb_get_state and lb_set_state move the unpadded state.
 * Size limits per lattice: sites < 2^31, and the planes of one velocity pair
 * below 4 GiB (2 x sites x element bytes in 3D, 3 x in D2Q9): 536M sites in
 * FP32, 268M in FP64, 1.07G in the 16-bit layouts.  Near contact needs every
 * axis >= 4 sites.
 * Errors: LB_EINVAL, LB_ENOMEM, LB_ENODEV, LB_EHIP.  *out is NULL on error. */
int lb_create(const lb_params* p, int n_channels, void* hip_stream, lb_handle** out);

/* Initialise channel `channel` (0 .. n_channels-1) with n droplets of the phase phi_in (+1: the
 * droplets are fluid A):
 *   phi(x) = phi_in * max_d tanh(2 (R_d - |x - c_d|) / width)
 * with minimum-image distances along periodic axes (2D ignores z), then
 * rho_A = rho0 (1 + phi)/2, rho_B = rho0 (1 - phi)/2 and f^k_i = f^eq_i(rho_k, u0)
 * (tanh interface profile of the free-energy section; Eq. disteq).
 * centres: host double[n][3] in site units; radii: host double[n].
 * n == 0 gives the uniform continuous phase.  Resets the step counter. */
int lb_init_droplets(lb_handle* h, int channel, int n, const double* centres,
                     const double* radii, double width, double phi_in);

/* Enqueue nsteps >= 0 time steps.  Each step pulls the populations, forms the
 * moments and phase field, the colour gradient and interface flags, the
 * near-contact force, collides (Guo-forced BGK, perturbation, recolouring)
 * and swaps buffers.  The macroscopic fields of the last step are kept for
 * lb_fields / lb_diagnostics.  With diag_every > 0 the watchdog runs every
 * diag_every steps (this synchronises) and a failure stops the loop with
 * LB_ENUMERIC. */
int lb_step(lb_handle* h, int nsteps);

/* Copy the fields selected by `mask` (LB_FIELD_* bits) of the last step (or of
 * the initial state) to dst[bit]: device pointers if dst_on_device, else host
 * pointers (then the call synchronises).  real = double for LB_F64, float
 * otherwise.  Labels are computed on demand. */
int lb_fields(lb_handle* h, int channel, unsigned mask, void* const* dst, int dst_on_device);

/* FP64 global diagnostics of the last step's fields, written to host out[8]:
 * [sum rho_A, sum rho_B, sum j_x, sum j_y, sum j_z, max |u|, droplet count,
 *  Laplace jump cs2 (<rho>_{phi > 0.9} - <rho>_{phi < -0.9}) (NaN if a side is empty)]
 * with j = rho u - F/2.  Synchronises. */
int lb_diagnostics(lb_handle* h, int channel, double out[8]);

/* Size in bytes of the raw state: per-colour layouts 2 * Q * N storage
 * elements f[k][i][s]; total layouts Q * N storage elements T[i][s] followed by
 * 4 * N floats (a, b_x, b_y, b_z as [4][s]).  An ensemble's state is its
 * channels' states concatenated in channel order. */
int lb_state_bytes(const lb_handle* h, size_t* bytes);
/* Copy the current post-collision state out / in, in the layout above (16-bit
 * modes hold the shifted values).  Host buffers when *_on_device == 0
 * (synchronises).  lb_set_state keeps the step counter; fields are available
 * again after the next step.  With LB_STREAM_IN_PLACE the state is always
 * given in this (canonical) layout: after an odd number of in-place steps
 * lb_get_state gathers it from the streamed slots (to a host buffer through a
 * one-plane staging buffer it allocates and frees). */
int lb_get_state(lb_handle* h, void* dst, size_t bytes, int dst_on_device);
int lb_set_state(lb_handle* h, const void* src, size_t bytes, int src_on_device);

/* Steps taken since the last lb_init_droplets. */
int lb_step_count(const lb_handle* h, long long* t);

/* Per-kernel timing for benchmarks.  Between lb_profile_begin and
 * lb_profile_end, lb_step records a hipEvent pair on the handle's stream
 * around every launch of the phase pass, of the collision pass and of the
 * read-once step's combine pass.  lb_profile_end synchronises and returns the
 * summed milliseconds and the launch counts of each (any pointer may be NULL). */
int lb_profile_begin(lb_handle* h);
int lb_profile_end(lb_handle* h, double* ms_phase, double* ms_collide, double* ms_combine, int* n_phase,
                   int* n_collide, int* n_combine);

/* Block until all work of the handle is done. */
int lb_sync(lb_handle* h);

/* Number of channels (1 for a single lattice). */
int lb_channel_count(const lb_handle* h, int* n);

/* Current / new ensemble launch configuration (single-lattice handles use
 * z_per_block and use_graph).  lb_set_tuning validates and rebuilds the work
 * lists (and drops a captured graph). */
int lb_get_tuning(const lb_handle* h, lb_tuning* t);
int lb_set_tuning(lb_handle* h, const lb_tuning* t);

/* Measure each candidate configuration for `steps` steps (hipEvents on the
 * handle's stream), keep the fastest and write it to *best.  results, if not
 * NULL, receives up to cap rows of {mode, z_per_block, use_graph, ms} as
 * doubles; *n_results the number of candidates.  The timed steps advance the
 * simulation: tune before lb_init_droplets or re-initialise afterwards. */
int lb_autotune(lb_handle* h, int steps, lb_tuning* best, double* results, int cap, int* n_results);

/* ---- Learned near-contact closure --------------------------------------------
 * The paper's outlook proposes learning near-contact forces from data
 * (Sec. VI.B.3).  The closure is a perceptron trained on rows the explicit
 * model generates:
 *   inputs (30)  phi on the 3x3x3 neighbourhood of an interface site, offsets
 *                (dx, dy, dz) in lexicographic order, index
 *                (dx+1) + 3 (dy+1) + 9 (dz+1) (wall ghosts mirrored, periodic
 *                axes wrapped), then the unit normal g/|g|
 *   network      tanh(W1 x + b1) (64), tanh(W2 h1 + b2) (64), W3 h2 + b3 (3)
 *   output       y, trained on F_nc / (nc_A |g|); the explicit force (A_h/2) g
 *                makes this target the normal n = g/|g| times A_h / (2 nc_A)
 *   force        the step applies the repulsive normal part of y, the form
 *                of the explicit force: F_nc = nc_A |g| max(0, y . n) n
 * Parameters are LB_MLP_PARAMS floats: W1 (64x30, row-major), b1 (64),
 * W2 (64x64), b2 (64), W3 (3x64), b3 (3).  Inference (in the collision pass
 * under LB_NC_MLP, and lb_mlp_infer) uses BF16 inputs, weights and hidden
 * values with FP32 accumulation on the matrix cores; training is FP32.  A site
 * uses the closure when all 30 inputs lie in [lo, hi] and |g| >= gmin (the
 * ranges of the training rows); other interface sites get the explicit scan.
 * With the closure, lb_fields' flags byte has bit 1 set where the network gave
 * the force and bit 2 where the explicit scan did.
 * Rows are LB_MLP_ROW floats: the 30 inputs, |g|, 0.  Targets are 3 floats. */
#define LB_MLP_PARAMS 6339
#define LB_MLP_ROW 32
#define LB_MLP_MAX_BATCH 65536

/* Training rows of the last step (which must have used LB_NC_EXPLICIT): one row
 * per interface site with |g| > 1e-12, target F_nc / (nc_A |g|).  Rows of
 * force-active sites come first, then force-free ones, each in site order
 * (x fastest).  rows (cap x LB_MLP_ROW) and targets (cap x 3) are device
 * pointers; at most cap rows are written.  *m_active / *m_free receive the
 * full counts (host pointers).  3D lattices only.  Synchronises. */
int lb_nc_collect(lb_handle* h, int channel, float* rows, float* targets, long long cap,
                  long long* m_active, long long* m_free);

/* lb_nc_collect for callers that cannot allocate device memory (code under
 * HIP graph capture, tight collection loops, harnesses that forbid
 * hipMalloc): the same rows, targets and counts, with the per-workgroup
 * counts and offsets in a static device array of the library (about 6 MB per
 * GPU, held until the process ends) and their scan done on the device.  Makes
 * no hipMalloc / hipFree call.  Lattices of at most 67,108,864 sites
 * (LB_EINVAL beyond).  Every call on one GPU uses that GPU's array: calls
 * that overlap on one GPU (handles on different streams or threads) race.
 * Synchronises. */
int lb_nc_collect_noalloc(lb_handle* h, int channel, float* rows, float* targets, long long cap,
                          long long* m_active, long long* m_free);

/* Network parameters (host pointers, n == LB_MLP_PARAMS).  Setting them
 * keeps the input ranges (initially empty: every site takes the explicit
 * scan until lb_mlp_set_ranges or lb_mlp_train sets them). */
int lb_mlp_set_weights(lb_handle* h, const float* theta, long long n);
int lb_mlp_get_weights(lb_handle* h, float* theta, long long n);

/* Input ranges of the closure (host pointers: lo[30], hi[30]). */
int lb_mlp_set_ranges(lb_handle* h, const float* lo, const float* hi, float gmin);
int lb_mlp_get_ranges(lb_handle* h, float* lo, float* hi, float* gmin);

/* Train from the current parameters with Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, fresh moments) on the mean squared error of the outputs: step t
 * (0 .. n_steps-1) uses rows order[t*batch .. (t+1)*batch).  rows (m x
 * LB_MLP_ROW), targets (m x 3), order (n_steps x batch int32) and loss_log
 * (n_steps floats, the batch loss before each update; may be NULL) are
 * device pointers.  The input ranges are then set from rows [0, m).
 * 1 <= batch <= LB_MLP_MAX_BATCH.  An order entry outside [0, m) is skipped
 * and the call returns LB_EINVAL after the run.  Synchronises. */
int lb_mlp_train(lb_handle* h, const float* rows, const float* targets, long long m, const int* order,
                 int n_steps, int batch, double lr, float* loss_log);

/* Loss and gradient of the mean squared error over rows [0, m) at the current
 * parameters (1 <= m <= LB_MLP_MAX_BATCH); grad (LB_MLP_PARAMS floats) and
 * loss (1 float) are device pointers.  Synchronises. */
int lb_mlp_gradient(lb_handle* h, const float* rows, const float* targets, long long m, float* grad, float* loss);

/* Network outputs (m x 3) for rows (m x LB_MLP_ROW), device pointers, with
 * the BF16 matrix-core evaluation of the collision pass.  Enqueued on the
 * handle's stream. */
int lb_mlp_infer(lb_handle* h, const float* rows, float* out, long long m);

/* Destroy a handle and free its device memory.  NULL is accepted. */
int lb_destroy(lb_handle* h);

/* Host-only: the velocity set this library uses.  q receives Q; c (int[Q][3]),
 * w (double[Q]), opp (int[Q]) and B (double[Q], perturbation coefficients)
 * may be NULL.  Needs no device. */
int lb_lattice_table(int lattice, int* q, int* c, double* w, int* opp, double* B);

/* Static text for a status code. */
const char* lb_error_string(int code);
/* Thread-local detail of the last failure (empty string if none). */
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
