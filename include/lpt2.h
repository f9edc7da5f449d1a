/*
 * lpt2.h -- C ABI of the MI355X (gfx950) library for FFT-based second-order
 * Lagrangian displacements in modified gravity.
 *
 * Method: Moretti, Mozzon, Monaco, Munari & Baldi (2019), "Fast numerical
 * method to generate halo catalogs in modified gravity (part I):
 * second-order Lagrangian Perturbation Theory".  The problem as the paper
 * states it (Sec. 3, procedure paragraph; Sec. 2.4): given a linear density
 * field on a regular periodic grid, a cosmology, a gravity model (mu(k,a) and
 * the expansion coefficients M_k) and an output time a, return the first-
 * and second-order displacement of every grid particle, with the
 * second-order growth factored as D2(k,a) times the GR spatial part.
 *
 * Conventions shared by every entry point
 *   - real fields are float or double [n][n][n], C order (x slowest, z
 *     fastest); particle (ix,iy,iz) sits at q = (ix,iy,iz) L/n;
 *   - displacement fields are [3][n][n][n] (component-major), in Mpc/h;
 *   - F is the unnormalised forward DFT, F^-1 carries 1/n^3;
 *     k = 2 pi m / L with m the signed FFT index;
 *   - the DC mode and every Nyquist plane (|m_i| = n/2) are zero in delta(k),
 *     S(k) and every k-space multiplier;
 *   - the precision of every field pointer is the plan's (LPT2_FP32: float,
 *     LPT2_FP64: double); growth factors, multipliers and twiddles are built
 *     in FP64 and rounded once;
 *   - field pointers are DEVICE pointers owned by the caller; host arrays are
 *     owned by the caller; the plan owns its workspace and tables;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - no entry point throws; each returns an lpt2_status, and the message of
 *     the last failure on a plan is available from lpt2_last_error().
 *   - a plan may be used by one host thread / one stream at a time; a
 *     concurrent call on the same plan returns LPT2_ESTATE.  Every call of a
 *     plan works in the plan's one workspace, so calls issued on different
 *     streams must be ordered by the caller (events or synchronisation);
 *     calls on one stream are ordered by the stream.
 */
#ifndef LPT2_H
#define LPT2_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lpt2_plan_s* lpt2_plan_t;        /* opaque; owns workspace and tables */

typedef enum {
  LPT2_OK = 0,
  LPT2_EINVAL = -1,        /* bad argument value or null pointer             */
  LPT2_EUNSUPPORTED = -2,  /* valid request this library does not implement  */
  LPT2_ENOMEM = -3,        /* device or host allocation failed               */
  LPT2_EDEVICE = -4,       /* HIP runtime or kernel launch error             */
  LPT2_ESTATE = -5         /* plan busy or used in the wrong order           */
} lpt2_status;

typedef enum { LPT2_FP64 = 0, LPT2_FP32 = 1 } lpt2_precision;

/* Gravity model (Sec. 2.2-2.4).  GR: mu = 1.  FR_HS: Hu-Sawicki f(R) with
 * n = 1, eq. mihusawicki for M1 = 3 m^2 and M2, mu(k,a) = 1 + (1/3)
 * (k^2/a^2)/(k^2/a^2 + m^2).  MU_CONST: constant mu (a test model with no
 * scalar mass; its growth starts on the EdS power-law mode). */
typedef enum { LPT2_GRAV_GR = 0, LPT2_GRAV_FR_HS = 1, LPT2_GRAV_MU_CONST = 2 } lpt2_gravity;

/* How D2(k,a) is obtained (Sec. 2.4 approximate factorisation; Sec. 3
 * triangle comparison; Sec. 5 eq. lcdm-fit).
 *   EDS      D2 = -3/7 D1^2
 *   T1       eq. full-d2 on the orthogonal isosceles triangle (k1 = k2, 90 deg)
 *   TRIANGLE eq. full-d2 on k1/k2 = tri_ratio at tri_theta_deg
 *   WINTHER  T1 geometry with D1(k)^2 in place of D1(k1) D1(k2)
 *   BOUCHET  D2 = -3/7 D1^2 Omega_m(a)^(-1/143)
 *   AUTO     chosen by the library once per a (Sec. 3): the first call at a
 *            that needs D2 (lpt2_displace, lpt2_backward, lpt2_autotune,
 *            lpt2_source_spectrum) runs lpt2_choose_factorisation's fit on
 *            the configuration's first realisation (n/2 shells, k <= 0.4
 *            h/Mpc) and synchronises; later calls use the chosen candidate. */
typedef enum {
  LPT2_D2_EDS = 0, LPT2_D2_T1 = 1, LPT2_D2_TRIANGLE = 2,
  LPT2_D2_WINTHER = 3, LPT2_D2_BOUCHET = 4, LPT2_D2_AUTO = 5
} lpt2_factorisation;

typedef enum { LPT2_SPEC_POWER = 0, LPT2_SPEC_RATIO = 1 } lpt2_spec_quantity;

typedef struct {
  int    n;               /* cells per side: 2^k in 8..512, 3*2^k in 24..768,
                             or 40, 56, 200, 400, 600, 700 (radices 5, 7)    */
  double box;             /* side length L in Mpc/h, > 0                       */
  double omega_m;         /* flat background: Omega_L = 1 - Omega_m           */
  double h;               /* BBKS shape parameter Gamma = Omega_m h            */
  double n_s;             /* primordial tilt                                   */
  double sigma8;          /* top-hat 8 Mpc/h normalisation of P(k) at a = 1    */
  int    gravity;         /* lpt2_gravity                                      */
  double fr0_abs;         /* |f_R0| > 0 for LPT2_GRAV_FR_HS                    */
  int    hs_n;            /* Hu-Sawicki n: must be 1                           */
  double mu_const;        /* mu for LPT2_GRAV_MU_CONST                         */
  int    factorisation;   /* lpt2_factorisation                                */
  double tri_ratio;       /* k1/k2 for LPT2_D2_TRIANGLE, > 0                   */
  double tri_theta_deg;   /* angle between k1 and k2, in (0, 180)              */
  int    nk_growth;       /* growth-table nodes, 2..1023 (default 256)         */
  double kmin, kmax;      /* node range in h/Mpc (default 1e-3, 10)            */
  double a_init;          /* ODE start (default 1e-3)                          */
  int    ode_steps;       /* fixed RK4 steps in ln a (default 4096)            */
  int    precision;       /* lpt2_precision                                    */
} lpt2_config;

/* Fill *cfg with the defaults above (GR, 32^3, L = 128, Omega_m = 0.3,
 * h = 0.7, n_s = 0.96, sigma8 = 0.8, EDS, FP64). */
void lpt2_config_default(lpt2_config* cfg);

/* Create a plan for n_cfgs grid configurations; counts[i] >= 1 realisations
 * of cfgs[i] (counts may be NULL for one realisation each).  Validates every
 * field on the host before any device work: n none of a power of two in
 * 8..512, three times one in 24..768 (the paper's 768^3 grid) or 40, 56,
 * 200, 400, 600, 700 (the paper's 200-700 Mpc/h boxes at 1 Mpc/h),
 * hs_n != 1 or an unknown precision -> LPT2_EUNSUPPORTED; box <= 0,
 * fr0_abs <= 0 for f(R), bad growth grid or null out -> LPT2_EINVAL.
 * Allocates, on the current device, the twiddles and a workspace of 16
 * half-spectrum slots per realisation of a batch: the realisations of one
 * configuration are transformed up to 64 at a time (fewer where 16 slots of
 * that many fields would pass 16 GiB), and every configuration has a region
 * of its own; and one small buffer: the shell binner's partial sums, the
 * lpt2_check_finite counter and, per configuration, the 16 tile-ticket words
 * of the column passes (zeroed here; every pass leaves them at zero).  On
 * failure *out is NULL. */
lpt2_status lpt2_plan(const lpt2_config* cfgs, int n_cfgs, const int* counts, lpt2_plan_t* out);

/* Release every device and host resource of the plan (NULL is a no-op). */
lpt2_status lpt2_destroy(lpt2_plan_t plan);

/* Total realisations held by the plan (sum of counts). */
int lpt2_realisations(lpt2_plan_t plan);

/* Grid size and precision of realisation r (0-based). */
lpt2_status lpt2_realisation_info(lpt2_plan_t plan, int r, int* n, int* precision);

/* Displacements at scale factor a > 0 (Sec. 3 procedure; eq. position):
 *   delta(k) = F[w] sqrt(P(k) n^3/V) mask,
 *   psi1     = F^-1[ i k D1(k,a)/k^2 delta(k) ],
 *   S        = sum_{i<j} (phi_,ii phi_,jj - phi_,ij^2),  phi_,ij = F^-1[-k_i k_j/k^2 delta(k)]
 *              (eq. second-ini, from the unevolved potential),
 *   psi2     = F^-1[ D2(k,a) (-i k/k^2) F[S] mask ].
 * noise[r], psi1[r], psi2[r] are device pointers for realisation r of the
 * plan (arrays of lpt2_realisations() entries): noise [n][n][n] unit white
 * noise; psi1 and psi2 [3][n][n][n] outputs.  The first call for a new a
 * builds its growth tables on `stream` (FP64 RK4 on the GPU, then per-|m|^2
 * tables) and caches them; later calls with the same a allocate nothing and
 * never synchronise.
 * Batches: each kernel of the chain covers a whole batch of realisations of
 * one configuration (one launch per pass, not per realisation).  With several
 * configurations each runs on a stream of the plan's own, forked from and
 * joined back into `stream`, so grids of different n overlap on the GPU.
 * In graph mode (lpt2_set_graph) the whole sequence is captured once per
 * (a, set of buffers) and later calls launch the graph on `stream`. */
lpt2_status lpt2_displace(lpt2_plan_t plan, double a, const void* const* noise,
                          void* const* psi1, void* const* psi2, void* stream);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * lpt2_displace of a one-realisation plan (noise, psi1, psi2 are single
 * device pointers), computed in a static device scratch of the library
 * instead of the plan's workspace, and allocating nothing: no hipMalloc,
 * hipFree, event creation or allocating library call on any path.
 *   - The scratch holds LPT2_NOALLOC_SLOT_BYTES for the 16 half-spectrum
 *     slots of the chain (16 n^3 reals: FP32 up to n = 96, FP64 up to
 *     n = 64) and LPT2_NOALLOC_TABLE_BYTES for growth and radial tables.
 *     A larger grid returns LPT2_EUNSUPPORTED; a plan of several
 *     realisations returns LPT2_EUNSUPPORTED.
 *   - Growth tables: the plan's cached tables at a if it has them (from an
 *     earlier lpt2_displace or lpt2_growth_table at that a), else they are
 *     rebuilt in the scratch on every call (the growth ODE runs each time).
 *   - An AUTO plan whose choice at a is not made returns LPT2_ESTATE.
 *   - Each GPU holds one copy of the scratch from the library's first plan
 *     on it until the process ends; every call on that GPU shares it and
 *     overwrites it (nothing in it needs to start at zero).  Calls that
 *     overlap on one GPU (other streams, other plans, other threads) race on
 *     the scratch: the caller must order them.
 *   - Results equal lpt2_displace's (the same kernels and tables); per-launch
 *     profiling is not recorded.  The tile tickets of the column passes, if
 *     a pass takes them, stay in the plan's small buffer (made with the
 *     plan, left at zero by every pass). */
#define LPT2_NOALLOC_SLOT_BYTES ((unsigned long)64 << 20)
#define LPT2_NOALLOC_TABLE_BYTES ((unsigned long)2 << 20)
lpt2_status lpt2_displace_noalloc(lpt2_plan_t plan, double a, const void* noise, void* psi1,
                                  void* psi2, void* stream);

/* Several output times from one source (Sec. 2.4: the factorised D2 makes
 * S(k) independent of a).  psi1 and psi2 at each of a[0..n_a) for every
 * realisation: the full chain runs once at a[0]; for a[1..] only the
 * first-order x pass (from the kept F[w]) and the second-order x pass (from
 * the kept F[S]) run again with that epoch's growth tables, with their y
 * and z passes.  Outputs are epoch-major: psi1[j * R + r] is realisation r
 * at a[j] (R = lpt2_realisations), [3][n][n][n] device arrays as in
 * lpt2_displace, whose results they equal.  n_a in 1..LPT2_MAX_EPOCHS.
 * Eager only (graph mode does not apply); growth tables as lpt2_displace. */
#define LPT2_MAX_EPOCHS 16
lpt2_status lpt2_displace_epochs(lpt2_plan_t plan, int n_a, const double* a,
                                 const void* const* noise, void* const* psi1,
                                 void* const* psi2, void* stream);

/* Graph mode on (enable != 0) or off.  In graph mode lpt2_displace captures
 * its launches (all grids and batches, with their fork and join) into a
 * hipGraph on a stream of the plan, instantiates it, caches it under
 * (a, noise/psi1/psi2 pointers) -- up to 8 graphs -- and launches it on the
 * caller's stream; a call with the same a and pointers only launches.
 * Turning graph mode off, changing tiles, or evicting growth tables
 * destroys the cached graphs (after a device synchronisation). */
lpt2_status lpt2_set_graph(lpt2_plan_t plan, int enable);

/* Tile widths (columns per workgroup) of configuration `grid`'s strided
 * passes: tiles[0] the single y (and x) FFT passes, tiles[1] the fused y
 * passes, tiles[2] the fused x passes.  lpt2_tile_options writes 9 ints,
 * widths[3*k + i] = option i of pass kind k: the widths giving 64-, 128- and
 * 256-byte row runs, clamped to the workgroup and LDS limits of that kind
 * (entries may repeat).  lpt2_set_tiles takes for each kind a width from its
 * list, or 0 for the default (option 1); anything else is LPT2_EINVAL.
 * Synchronises if the tiles change. */
lpt2_status lpt2_get_tiles(lpt2_plan_t plan, int grid, int* tiles);
lpt2_status lpt2_set_tiles(lpt2_plan_t plan, int grid, const int* tiles);
lpt2_status lpt2_tile_options(lpt2_plan_t plan, int grid, int* widths);

/* Tile tuner: for every configuration, runs its batches at a on the given
 * buffers (same meaning as lpt2_displace; their contents are overwritten)
 * under every combination of the offered tile widths, timing each with HIP
 * events on `stream` (one warm run, minimum of three), and keeps the fastest.
 * cache_path (may be NULL) names a text file: an entry for the same device
 * architecture, precision, n and batch size is used without timing, and new
 * results are appended as lines
 *   lpt2-tiles <arch> <fp32|fp64> <n> <batch> <tile0> <tile1> <tile2>
 * Synchronises. */
lpt2_status lpt2_autotune(lpt2_plan_t plan, double a, const void* const* noise,
                          void* const* psi1, void* const* psi2, const char* cache_path,
                          void* stream);

/* Test entry (a density field in place of white noise): psi1 and psi2 of
 * realisation 0's grid for the given real-space density contrast delta
 * ([n][n][n] device, the plan's precision): delta(k) = F[delta] mask, then as
 * lpt2_displace (no sqrt(P) shaping).  Growth and radial tables are cached
 * per a beside the white-noise ones.  An AUTO configuration must have made
 * its choice at a (LPT2_ESTATE otherwise). */
lpt2_status lpt2_displace_delta(lpt2_plan_t plan, double a, const void* delta, void* psi1,
                                void* psi2, void* stream);

/* Matter power spectrum of the displaced particles of realisation 0: their
 * cloud-in-cell density (as lpt2_paint_cic) is transformed on the grid and
 * q = V |F[delta]/n^3|^2 is binned in nbins shells as in
 * lpt2_source_spectrum (integer-exact shells of width k_Nyq/nbins, DC and
 * modes at or beyond k_Nyq left out).  flags (an OR of):
 *   LPT2_POWER_DECONVOLVE  divide each mode by W^2, W = prod_i sinc^2(pi m_i/n)
 *                          the CIC window;
 *   LPT2_POWER_INTERLACE   interlacing: the particles are painted a second
 *                          time moved by half a cell along every axis, that
 *                          transform is multiplied by exp(i pi (m_x+m_y+m_z)/n)
 *                          and averaged with the first, which cancels the
 *                          alias images with an odd index sum.
 * Other bits are LPT2_EINVAL.  Host arrays of nbins values; the float atomics
 * of the painting make the last bits vary from run to run.  nbins in 1..512.
 * Synchronises. */
#define LPT2_POWER_DECONVOLVE 1
#define LPT2_POWER_INTERLACE 2
lpt2_status lpt2_matter_power(lpt2_plan_t plan, const void* psi1, const void* psi2, int nbins,
                              int flags, double* k_mean, double* count, double* mean,
                              double* std_dev, void* stream);

/* Eulerian particle positions (eq. position): x = (q + psi1 + psi2) mod L for
 * the particles of realisation r's grid, q = (ix, iy, iz) L/n; psi1, psi2
 * and pos are [3][n][n][n] device arrays in the plan's precision (pos may
 * alias neither input).  Asynchronous on `stream`. */
lpt2_status lpt2_positions(lpt2_plan_t plan, int r, const void* psi1, const void* psi2, void* pos,
                           void* stream);

/* Shell-binned spectrum of the source for realisation 0 (Sec. 3: bin a
 * per-mode quantity in k, report mean and 1-sigma scatter).
 * quantity = LPT2_SPEC_POWER: q = V |S(k)/n^3|^2 of the displacement path's
 * source.  quantity = LPT2_SPEC_RATIO: q = Re(S_MG conj S_GR)/|S_GR|^2 with
 * S_MG = S1+S2+S3+S4 of eqs. full, s1-s4 (evolved with D1(k,a); S1 with the
 * term -mu(k) F[phi_ij phi_ij] that its GR limit requires) and S_GR from the
 * unevolved field; modes with S_GR = 0 are left out.
 * nbins shells of width k_Nyq/nbins, integer-exact shell index
 * isqrt(|m|^2 nbins^2 / (n/2)^2); weight 2 for 0 < m_z < n/2, else 1; DC and
 * modes beyond the last shell are left out.  Writes nbins values to each host
 * array: mean k, weighted count, mean q, population std of q (zeros for an
 * empty shell).  Synchronises `stream` before returning.  nbins in 1..512. */
lpt2_status lpt2_source_spectrum(lpt2_plan_t plan, double a, const void* noise, int nbins,
                                 int quantity, double* k_mean, double* count,
                                 double* mean, double* std_dev, void* stream);

/* Analytic MG/GR source ratio of triangle configurations at the wavenumbers
 * k[0..nk) (Sec. 3, triangle comparison): R(k) = D1(k1) D1(k2) B / (D1_GR^2
 * (1 - cos^2 theta)), B the braced factor of eq. full-d2; winther != 0 uses
 * D1(k)^2.  Host arrays; growth tables as for lpt2_displace. */
lpt2_status lpt2_triangle_ratio(lpt2_plan_t plan, double a, double ratio, double theta_deg,
                                int winther, const double* k, int nk, double* out);

/* Candidate triangles of the factorisation choice (Sec. 3, triangle
 * comparison), in this order: T1 (k1 = k2, 90 deg), T2 (k1 = k2, 80 deg),
 * k1 = k2 at 70 deg, equilateral (60 deg), squeezed (k1/k2 = 1e-3, 90 deg),
 * k1 = 2 k2 at 80 and at 70 deg, and Winther's (D1(k)^2 in place of
 * D1(k1) D1(k2), 90 deg).  lpt2_factorisation_candidate writes candidate
 * i's name (static storage), k1/k2 ratio, angle and Winther flag (any
 * pointer may be NULL); i out of range -> LPT2_EINVAL. */
int         lpt2_factorisation_candidates(void);
lpt2_status lpt2_factorisation_candidate(int i, const char** name, double* ratio,
                                         double* theta_deg, int* winther);

/* Factorisation choice (Sec. 3): the binned ratio S_MG/S_GR of realisation 0
 * at a, as lpt2_source_spectrum with LPT2_SPEC_RATIO and nbins shells, is
 * compared with each candidate's lpt2_triangle_ratio at the shell mean
 * wavenumbers; the cost of a candidate is sum_shells count (mean - R)^2 over
 * the populated shells with 0 < k_mean <= kcut (h/Mpc).  Writes the index of
 * the cheapest candidate to *best and, if costs is not NULL, every cost to
 * costs[0..lpt2_factorisation_candidates()).  apply != 0 makes the chosen
 * candidate realisation 0's configuration's D2: for an AUTO configuration
 * its choice at this a; for any other, its factorisation at every a (cached
 * growth tables and captured graphs are dropped and rebuilt on the next
 * call).  nbins in 1..512, kcut > 0; no populated shell below kcut ->
 * LPT2_EINVAL.  Synchronises. */
lpt2_status lpt2_choose_factorisation(lpt2_plan_t plan, double a, const void* noise, int nbins,
                                      double kcut, int apply, int* best, double* costs,
                                      void* stream);

/* The candidate an AUTO configuration `grid` uses at a (index as in
 * lpt2_factorisation_candidate), or -1 if not chosen yet (or not AUTO). */
lpt2_status lpt2_auto_choice(lpt2_plan_t plan, int grid, double a, int* candidate);

/* Counts the non-finite values (NaN, +-inf) of a device array of `count`
 * reals in the plan's precision (a noise field before lpt2_displace, say:
 * the displacement entry points do not scan their inputs, and one
 * non-finite noise value spreads through every transform to all outputs).
 * Synchronises `stream`.  *nonfinite receives the count; the call returns
 * LPT2_EINVAL when it is not zero and LPT2_OK otherwise. */
lpt2_status lpt2_check_finite(lpt2_plan_t plan, const void* field, long long count, long long* nonfinite,
                              void* stream);

/* Vector-Jacobian product of lpt2_displace: given g_psi1[r], g_psi2[r]
 * (device, [3][n][n][n]) returns g_noise[r] = d/dw sum(g_psi1 psi1 + g_psi2 psi2)
 * (device, [n][n][n]).  phi_,ij are recomputed from noise[r], not stored.
 * Each linear block F^-1 M F is transposed as F^-1 conj(M) F; the quadratic
 * source is differentiated by the product rule.  Same allocation and
 * synchronisation rules as lpt2_displace. */
lpt2_status lpt2_backward(lpt2_plan_t plan, double a, const void* const* noise,
                          const void* const* g_psi1, const void* const* g_psi2,
                          void* const* g_noise, void* stream);

/* Cloud-in-cell density of the displaced particles of realisation 0:
 * delta[g] = sum_p prod_axes max(0, 1 - |x_p - g L/n|/(L/n)) - 1, periodic,
 * x_p = q_p + psi1_p + psi2_p (eq. position).  The density contrast of the
 * displaced particles follows from mass conservation (eq. deltajacobian:
 * each particle carries the mass of its Lagrangian cell); painting the
 * particles on the mesh is the discrete form used here, which conserves the
 * total mass exactly.  delta is a device [n][n][n] output.  Non-finite
 * positions, and positions more than 2^30 cells from the origin, are not
 * painted.  FP32 plans sum each workgroup's weights in 32-bit fixed point
 * (step 1/(2^22 - 1), exact integer sums) and add them to delta with float
 * atomics; FP64 plans use double atomics throughout.  The order of the
 * atomics, and so the last bits of delta, vary from run to run. */
lpt2_status lpt2_paint_cic(lpt2_plan_t plan, const void* psi1, const void* psi2,
                           void* delta, void* stream);

/* Transpose of lpt2_paint_cic at the same displacements: g_psi [3][n][n][n]
 * = d/dx_p sum_g g_delta[g] delta[g] (the same array serves as the gradient
 * for psi1 and psi2).  Deterministic (a gather). */
lpt2_status lpt2_paint_cic_backward(lpt2_plan_t plan, const void* psi1, const void* psi2,
                                    const void* g_delta, void* g_psi, void* stream);

/* Growth tables at a (host copies, nk_growth doubles each): node k, D1(k,a),
 * D2(k,a), normalised so that D1(k -> 0, a = 1) = 1 (Sec. 2.4).  Synchronises. */
lpt2_status lpt2_growth_table(lpt2_plan_t plan, double a, double* k, double* d1, double* d2);

/* Test entry: 3D real FFT of realisation 0's grid in the library's internal
 * spectral layout.  direction = -1: in is a real [n][n][n] field, out is
 * complex [n][n][n/2] (interleaved re,im; the m_z = n/2 plane is not stored)
 * holding the unnormalised F.  direction = +1: in is complex [n][n][n/2],
 * taken as the half spectrum of a real field with a zero m_z = n/2 plane and
 * real m_z = 0 column values; out is the real field n^3 F^-1 (unnormalised).
 * Device pointers; `in` is left unchanged. */
lpt2_status lpt2_fft3d(lpt2_plan_t plan, int direction, const void* in, void* out, void* stream);

/* Per-kernel timing with HIP events on the stream each kernel is launched
 * on.  enable != 0 records an event pair around every kernel launch of later
 * eager calls (not inside a graph capture); the counters accumulate until
 * lpt2_profile_reset.  lpt2_profile_get reports entry i (0-based,
 * i < lpt2_profile_count), one per (launch site, bytes per launch): its name
 * (static storage), launches, summed milliseconds and algorithmic bytes per
 * launch (the compulsory reads and writes of that kernel over its whole
 * batch).  Synchronises. */
lpt2_status lpt2_profile_enable(lpt2_plan_t plan, int enable);
lpt2_status lpt2_profile_reset(lpt2_plan_t plan);
int         lpt2_profile_count(lpt2_plan_t plan);
lpt2_status lpt2_profile_get(lpt2_plan_t plan, int i, const char** name, long long* launches,
                             double* total_ms, double* bytes_per_launch);

/* Bytes of device workspace held by the plan. */
long long lpt2_workspace_bytes(lpt2_plan_t plan);

const char* lpt2_strerror(lpt2_status status);
const char* lpt2_last_error(lpt2_plan_t plan);   /* "" if none; NULL plan: last plan-less error */

#ifdef __cplusplus
}
#endif
#endif /* LPT2_H */
