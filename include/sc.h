/*
 * sc.h -- C ABI of the MI355X (gfx950) Stratton-Chu mirror-focusing library.
 *
 * The library evaluates the physical-optics (POA) Stratton-Chu diffraction
 * integrals of a field reflected off a parabolic mirror, in the
 * Stokes-converted form of Dumont et al. (arXiv:1609.08146, Sec. II,
 * eq. stratton-chu-poa-og):
 *
 *   E'(r',k) = 2 SS { ik (n x B_inc) g + (n . E_inc) grad g } dS
 *              - (2/ik) O grad g [ n x (n x B_inc) ] . dl
 *   B'(r',k) = 2 SS (n x B_inc) x grad g dS,      g = e^{ik|r-r'|} / (4 pi |r-r'|),
 *
 * with the gradient taken on the mirror variable r, by plain tensor-product
 * quadrature over the mirror (Gauss-Legendre in r, trapezoid rule in phi;
 * Sec. III-C), for every observation point and every frequency, and then
 * transforms the spectral field to the time domain with the semi-discrete
 * Fourier sum F(t) = sum_n F_n e^{-i k_n t} dk (Sec. III-B,
 * eq. impl.semiDiscreteFFT).
 *
 * Units and conventions: c = 1 (Lorentz-Heaviside), k = omega, time factor
 * e^{-ikt}; any consistent length unit; t is c*t.  The mirror is the
 * paraboloid z = r^2/(4f) - f with its focus at the origin (Sec. III-C-1);
 * the incident beam travels along -z (Sec. III-A).  The unnormalised normal
 * n~ = (-x/2f, -y/2f, 1) points from the mirror toward the focus and the
 * incoming beam, so that n dS = n~ r dr dphi.  Results are the REFLECTED
 * field only.  Observation points on the mirror surface are outside the
 * method's domain (g is singular there); they are not checked.
 *
 * Complex arrays are interleaved (re, im) pairs: complex128 = 2 doubles,
 * complex64 = 2 floats.
 *
 * Memory and streams: every entry point enqueues its GPU work on the
 * context's HIP stream.  Pointers flagged on_device = 1 are device pointers
 * on the context's device; they must stay valid until the stream work that
 * reads or writes them has completed (sc_ctx_synchronize).  Host pointers
 * (on_device = 0) are read before the call returns; host outputs are complete
 * when the call returns.  The library never retains or frees caller memory.
 *
 * Errors: every entry point returns an sc_status; nothing throws across the
 * ABI.  On a non-OK status, sc_last_error() returns a thread-local message.
 * A failed call leaves the object in its previous valid state unless stated.
 *
 * Threads: a context and its problems must not be used from two threads at
 * once; the serving API below is the thread-safe front end.
 */
#ifndef SC_H
#define SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_ctx sc_ctx;
typedef struct sc_prob sc_prob;
typedef struct sc_server sc_server;

typedef enum {
    SC_OK = 0,
    SC_E_INVAL = -1,        /* bad argument (size, value, null pointer)            */
    SC_E_NOMEM = -2,        /* device or host allocation failed / over HBM budget   */
    SC_E_DEVICE = -3,       /* HIP runtime error                                    */
    SC_E_STATE = -4,        /* call out of order (e.g. evaluate before inputs)      */
    SC_E_UNSUPPORTED = -5,  /* option not available                                 */
    SC_E_TIMEOUT = -6,      /* serving: wait timed out (request still queued)       */
    SC_E_CANCELLED = -7,    /* serving: request was cancelled                       */
    SC_E_REJECTED = -8      /* serving: request can never fit the HBM budget        */
} sc_status;

/* Arithmetic of the quadrature.
 *  SC_FP64       all per-pair arithmetic in FP64; node phase k|r_s| in double-double.
 *                Output complex128.
 *  SC_FP32_SPLIT the large phase k|r_s| (up to ~1e6 rad) is folded into the
 *                per-(k,node) tables in double-double/FP64 and reduced mod 2pi;
 *                the per-pair remainder k(|r_s - r'| - |r_s|) is formed without
 *                cancellation and evaluated in FP32; FP32 sums over blocks of
 *                512 nodes, added into per-chunk running sums, and the chunk
 *                sums added in FP64.  Output complex64.
 *  SC_FP32       naive FP32: per-pair phase k|r_s - r'| in FP32 (an ablation;
 *                loses accuracy once k|r_s| >> 1e3).  Output complex64.
 */
typedef enum { SC_FP64 = 0, SC_FP32_SPLIT = 1, SC_FP32 = 2 } sc_precision;

const char *sc_last_error(void);
const char *sc_version(void);

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `stream` is a hipStream_t to use,
 * or NULL for a library-owned stream (default priority).  */
sc_status sc_ctx_create(int device, void *stream, sc_ctx **out);
/* Destroy a context.  SC_E_STATE (and nothing is freed) while problems
 * created on it are still alive.                                           */
sc_status sc_ctx_destroy(sc_ctx *ctx);
/* Wait for all work enqueued on the context's stream.                       */
sc_status sc_ctx_synchronize(sc_ctx *ctx);
/* Record HIP events around each kernel phase (see sc_get_timing).           */
sc_status sc_ctx_set_profiling(sc_ctx *ctx, int enable);

/* Per-phase device times of the most recent evaluate / to_time on a problem,
 * in milliseconds, measured with HIP events on the context's stream
 * (valid once the stream has completed; needs profiling enabled). */
typedef struct {
    double prep_ms;      /* incident/node table preparation (last set_incident*) */
    double quad_ms;      /* the quadrature kernel (all tiles)                     */
    double reduce_ms;    /* split-K reduction into the output                     */
    double time_ms;      /* the semi-discrete time transform                      */
    int64_t evals;       /* obs x freq x surface nodes of the last evaluate       */
    int64_t tiles;       /* quadrature tiles of the last evaluate                 */
    int32_t chunk;       /* node chunk of the last evaluate (fixes its bits)      */
} sc_timing;
sc_status sc_get_timing(const sc_prob *p, sc_timing *out);

/* Quadrature launch shape.  Only `chunk` changes the floating-point
 * summation order (and therefore the last bits of results); the other
 * fields change speed only.  Zero fields mean "library default": 1 point per
 * lane, 4 waves per workgroup, chunks of 2048 nodes, the resident limit of
 * workgroups, and frequencies per lane by table layout (4 with the factored
 * current in the FP32 forms, else 2).                                       */
typedef struct {
    int obs_per_lane;    /* 1 or 2 observation points per lane                    */
    int waves_per_block; /* 1, 2 or 4 waves of 64 lanes per workgroup             */
    int chunk;           /* mirror nodes per split-K chunk (multiple of 64)        */
    int blocks_per_cu;   /* persistent workgroups per compute unit (0 = max)       */
    int freq_per_lane;   /* 1, 2 or 4 frequencies per lane sharing one geometry
                            (obs_per_lane x freq_per_lane <= 4, not 2 x 4)        */
} sc_launch;
/* Fix the launch shape for a problem (overrides the context's tuned value). */
sc_status sc_set_launch(sc_prob *p, const sc_launch *launch);
/* The launch shape an evaluation of `p` in precision `prec` uses now (the
 * problem's override, else the context's tuned entry for its size bucket,
 * else the library default), every field filled in.  `out` is host memory.
 * SC_E_INVAL for NULL arguments or an unknown precision.                   */
sc_status sc_get_launch(const sc_prob *p, sc_precision prec, sc_launch *out);
/* Time candidate launches on problem `p` (quadrature plus reduction, best of
 * two runs each) and store the fastest in the context's cache, keyed by
 * (precision, table layout, size buckets of n_obs, n_k and nodes): first the
 * kernel shape and waves per workgroup at the library's chunk, then the chunk
 * (512 ... 16384 nodes) and workgroups per CU.  A tuned chunk sets the
 * summation order, so every problem of the bucket then gets that chunk's bits
 * (alone and in batches alike).  `budget_ms` bounds the time spent (0 = 20 s);
 * *best (may be NULL) receives the winner.                                  */
sc_status sc_autotune(sc_prob *p, sc_precision prec, double budget_ms, sc_launch *best);
/* The launch of sc_evaluate_batch in precision `prec`: the kernel shape,
 * waves per workgroup and workgroups per CU of the one persistent launch, and
 * `chunk` = 0 (each problem keeps its own) or a chunk for every problem of the
 * batch that does not fix one with sc_set_launch.  NULL clears it, and the
 * batch then takes the library's shape for the table layout that carries most
 * of its evaluations.                                                        */
sc_status sc_set_batch_launch(sc_ctx *ctx, sc_precision prec, const sc_launch *launch);
/* Time candidate batch launches on the batch `probs[0..n)` (pass a
 * representative part of a large batch: every candidate evaluates all of
 * them) and keep the fastest as the context's batch launch for `prec`: first
 * the kernel shape and waves per workgroup, then one chunk for the batch (or
 * each problem's own) and workgroups per CU.  A problem evaluated in a batch
 * with a tuned chunk gives its alone result at that chunk (sc_set_launch).  */
sc_status sc_autotune_batch(sc_ctx *ctx, sc_prob *const *probs, int n, sc_precision prec, double budget_ms,
                            sc_launch *best);
/* Load / save the context's tuning cache (plain text).                     */
sc_status sc_autotune_load(sc_ctx *ctx, const char *path);
sc_status sc_autotune_save(sc_ctx *ctx, const char *path);

/* ------------------------------------------------------------------ problem */

sc_status sc_prob_create(sc_ctx *ctx, sc_prob **out);
/* Frees every device buffer the problem owns; never caller memory.          */
sc_status sc_prob_destroy(sc_prob *p);

/* Mirror z = r^2/(4f) - f, r in [0, r_max] (Sec. III-C-1): n_r Gauss-Legendre
 * nodes in r on [0, r_max] and n_phi trapezoid nodes phi_j = 2 pi j / n_phi,
 * plus n_phi rim nodes at r = r_max for the line integral.  Node order:
 * surface node (i, j) at index i*n_phi + j, then the rim nodes.
 * f > 0, r_max > 0, 1 <= n_r, 1 <= n_phi, (n_r+1)*n_phi < 2^31 (SC_E_INVAL).
 * Invalidates the incident tables and results.                             */
sc_status sc_set_mirror(sc_prob *p, double f, double r_max, int n_r, int n_phi);
/* A general mirror given by its own quadrature, for surfaces other than the
 * built-in paraboloid (the method holds for any perfectly conducting
 * surface, Sec. II; Sec. III-C-1 discusses why the paraboloid needs no
 * sub-wavelength mesh and other shapes may).  Host arrays:
 *   xyz [n_surf][3]      surface nodes;
 *   ndS [n_surf][3]      area-weighted normals n dS (quadrature weight times
 *                        the normal, pointing from the mirror toward the
 *                        focus and the incoming beam);
 *   rim_xyz [n_rim][3]   nodes of the boundary curve;
 *   rim_n [n_rim][3]     the surface normal there (direction only);
 *   rim_dl [n_rim][3]    oriented line elements dl (weight times tangent,
 *                        right-handed about the normal: counter-clockwise seen
 *                        from the beam on the outer edge, clockwise on holes).
 * n_rim = 0 drops the line integral (a surface without boundary).  Replaces
 * the mirror and invalidates the tables.  The split form is accurate when the
 * observation points lie near the origin (|r'| << |r_s|); the node phase is
 * folded as for the paraboloid.  Where the folded integrand oscillates over
 * the surface (any shape but the paraboloid), its terms cancel in the sum, and
 * per-term rounding of the FP32-split form weighs by the ratio
 * sum |term| / |sum of terms| (about 70 at the focus of an ellipsoidal cap
 * whose folded phase spans 330 rad, where FP32-split measured 2e-5 to 6e-5
 * of the field peak against 1e-6 on the paraboloid): use SC_FP64 there.
 * SC_E_INVAL for bad sizes or non-finite data.                               */
sc_status sc_set_surface(sc_prob *p, int n_surf, const double *xyz, const double *ndS, int n_rim,
                         const double *rim_xyz, const double *rim_n, const double *rim_dl);
/* Number of surface nodes (n_r*n_phi) and rim nodes (n_phi).                */
sc_status sc_get_num_nodes(const sc_prob *p, int *n_surface, int *n_rim);
/* The mirror's quadrature (Sec. III-C-1: the tensor-product rule over the
 * mirror's cylindrical parametrisation), copied to host arrays so that a
 * caller can tabulate its incident field on the nodes (sc_set_incident); any
 * pointer may be NULL:
 *   xyz    [(n_r+1)*n_phi][3] positions (surface nodes, then rim),
 *   normal [(n_r+1)*n_phi][3] unnormalised normals n~ (n dS = n~ weight),
 *   weight [(n_r+1)*n_phi]    surface weights w_r(i) r_i 2pi/n_phi, then the rim
 *                             weights 2pi/n_phi (the rim tangent is dr_s/dphi).
 * For a general surface (sc_set_surface): the caller's nodes, its n dS as the
 * normal with weight 1, and the boundary's normals with weight 1.
 * SC_E_STATE without a mirror.                                              */
sc_status sc_get_nodes(const sc_prob *p, double *xyz, double *normal, double *weight);

/* Size limits (grid dimensions of the per-frequency and time kernels).      */
#define SC_MAX_FREQUENCIES 65535
#define SC_MAX_TIMES 524280

/* The frequency samples of the spectral field (Sec. III-B: the pulse is
 * handled as a sum over frequency components, each evaluated on its own):
 * wavenumbers k_n = omega_n > 0 (c = 1), 1 <= n_k <= SC_MAX_FREQUENCIES, in
 * any order and spacing (sc_to_time needs a uniform grid, sc_to_time_at does
 * not).  k: host [n_k].  SC_E_INVAL for non-positive or non-finite values.
 * Invalidates the incident tables and results.                              */
sc_status sc_set_frequencies(sc_prob *p, const double *k, int n_k);

/* Incident field on the mirror nodes (Sec. III-A): E and B are complex128
 * [n_k][(n_r+1)*n_phi][3] in sc_get_nodes order, rim row included, and hold the
 * full spectral field at each node (propagation phase such as e^{-ikz},
 * spectral amplitude and any spectral phase, Sec. III-B).  The physical-
 * optics current J = 2 n x B_inc (Sec. II, eq. poa) and the charge term
 * n . E_inc are formed on the device.  Needs mirror and frequencies
 * (SC_E_STATE).  Device tables of ~64 B per (k, node) are kept resident.    */
sc_status sc_set_incident(sc_prob *p, const double *E, const double *B, int on_device);
/* Built-in collimated beams travelling along -z, evaluated on the device at
 * every node and frequency (Sec. III-A; the radially polarised beam is the
 * one of the numerical checks of Sec. IV-A, the linearly polarised one that
 * of Sec. IV-B).  With psi = G e^{-ikz}:
 *   SC_BEAM_LINEAR, G = exp(-(x^2+y^2)/w0^2), in the frame where the
 *     polarisation is along x (pol_angle rotates the beam about z):
 *     consistent = 0: E = x psi, B = (-z) x E = -y psi
 *     consistent = 1: B = psi (0, -1, -2iy/(k w0^2)), E = (i/k) curl B
 *     w0 = +inf gives a plane wave;
 *   SC_BEAM_RADIAL, G = exp(-r^2/w0^2) / w0:
 *     E = psi (x, y, c), B = psi (y, -x, 0);
 *   SC_BEAM_AZIMUTHAL: E = psi (-y, x, 0), B = psi (x, y, c);
 *   c = (2i/k)(r^2/w0^2 - 1) when consistent (then E = (i/k) curl B for the
 *   radial and B = (-i/k) curl E for the azimuthal beam), else c = 0
 *   (B = (-z) x E).  The cylindrical beams need a finite w0 and do not
 *   depend on pol_angle.  spectrum: complex128 [n_k] amplitudes (NULL = 1). */
typedef enum { SC_BEAM_LINEAR = 0, SC_BEAM_RADIAL = 1, SC_BEAM_AZIMUTHAL = 2 } sc_beam;
sc_status sc_set_incident_beam(sc_prob *p, int beam, double w0, double pol_angle,
                               const double *spectrum, int consistent);
/* Laguerre-Gauss mode sets (Sec. III-A: the Laguerre-Gauss modes of the
 * paraxial wave equation are the expansion basis of the incident linearly and
 * radially polarised beams).  Each mode is taken in its waist cross-section
 * and carried along -z without diffraction (a collimated beam, as the
 * Gaussians above; the divergence is neglected, as Sec. III-A argues):
 *   u_{p,l}(r, phi) = C_{p,l} (sqrt(2) r / w0)^|l| L_p^|l|(2 r^2 / w0^2)
 *                     exp(-r^2 / w0^2) e^{i l phi},
 *   C_{p,l} = sqrt(2 p! / (pi (p + |l|)!)) / w0  (unit integral of |u|^2 over
 * the plane), L_p^a the generalized Laguerre polynomial.  A mode carries
 * complex amplitudes ex, ey of its x- and y-polarised parts, and
 *   E = amp_n e^{-ikz} sum_m (ex_m x + ey_m y) u_m,
 *   B = (-z) x E = amp_n e^{-ikz} sum_m (ey_m x - ex_m y) u_m
 * (transverse fields; amp_n from `spectrum`, complex128 [n_k], NULL = 1).
 * LG_{0,0} with ex = 1 is sqrt(2/pi)/w0 times the literal Gaussian, and
 * (LG_{0,1} + LG_{0,-1}) / (2 sqrt 2 C_{0,1}) in x plus
 * (LG_{0,1} - LG_{0,-1}) / (2i sqrt 2 C_{0,1}) in y is the radially polarised
 * beam above.  Whether the tables factor (sc_set_factoring) is decided from
 * the tables as for any field: modes sharing one linear polarisation, and
 * the radial combination above, keep one real current direction per node and
 * factor; a circularly polarised part generally does not.
 * 1 <= n_modes <= SC_MAX_LG_MODES, 0 <= p <= SC_MAX_LG_INDEX,
 * |l| <= SC_MAX_LG_INDEX, finite amplitudes, 0 < w0 < inf (SC_E_INVAL);
 * needs mirror and frequencies (SC_E_STATE).  `modes` is host memory.      */
#define SC_MAX_LG_MODES 64
#define SC_MAX_LG_INDEX 64
typedef struct {
    int p;          /* radial index                                  */
    int l;          /* azimuthal index (either sign)                 */
    double ex[2];   /* complex amplitude (re, im) of the x part      */
    double ey[2];   /* complex amplitude (re, im) of the y part      */
} sc_lg_mode;
sc_status sc_set_incident_lg(sc_prob *p, const sc_lg_mode *modes, int n_modes, double w0,
                             const double *spectrum);
/* The linearly polarised Gaussian: sc_set_incident_beam(p, SC_BEAM_LINEAR, ...). */
sc_status sc_set_incident_gaussian(sc_prob *p, double w0, double pol_angle,
                                   const double *spectrum, int consistent);

/* Power carried by each frequency component of the incident field through
 * the mirror aperture (Sec. III-B, the Poynting integral that fixes the
 * energy of a component):
 *   P[n] = 4 pi SS Re(E_n x B_n^*) . dA,   dA = -z dx dy over r <= r_max
 * (the beam travels along -z), by the same quadrature as the mirror integrals
 * projected on the aperture plane (surface weights w_r r dphi; rim nodes do
 * not enter).  Computed on the device whenever the incident field is set and
 * kept up to date by sc_scale_spectrum / sc_normalize_energy.
 * P: host [n_k].  SC_E_STATE without an incident field.                     */
sc_status sc_get_incident_power(const sc_prob *p, double *P);
/* Multiply frequency n of the incident field by factor[n] (complex128 [n_k],
 * host): a spectral amplitude and phase, e.g. a chirp e^{i phi(omega)}
 * (Sec. III-B).  Earlier results are discarded; P[n] scales by |factor[n]|^2.
 * SC_E_STATE without an incident field; SC_E_INVAL for non-finite factors. */
sc_status sc_scale_spectrum(sc_prob *p, const double *factor);
/* Energy normalisation of the incident spectrum (Sec. III-B, eqs.
 * normalizationAmplitude and totalEnergy).  eps: host [n_k] power spectrum
 * samples eps(k_n) >= 0 (energy per unit k).  If e_tot > 0 they are first
 * rescaled so that sum_n eps_n dk = e_tot (the discrete total-energy
 * condition; dk > 0 required), else taken as given.  Frequency n is then
 * multiplied by E0_n = sqrt(eps_n / P[n]) with P[n] the current incident
 * power, so that afterwards sc_get_incident_power returns eps_n.  A sample
 * with eps_n = 0 removes its component.  SC_E_INVAL for negative or
 * non-finite eps, or a component with eps_n > 0 but no power (P[n] <= 0).  */
sc_status sc_normalize_energy(sc_prob *p, const double *eps, double e_tot, double dk);

/* Table storage.  keep_fp64 = 1 (default) keeps the FP64 tables (64 B per
 * (k, node)) so every precision can be evaluated; keep_fp64 = 0 casts them to
 * the FP32 split tables (32 B per record) as soon as they are built and frees
 * them, halving resident memory; SC_FP64 evaluation then fails with
 * SC_E_STATE until the incident field is set again with keep_fp64 = 1.     */
sc_status sc_set_table_storage(sc_prob *p, int keep_fp64);

/* Factored current for SC_FP32_SPLIT and SC_FP64.  The surface current of the integrand
 * (Sec. II: J = n x B_inc, with the quadrature weight and the node phase
 * folded in) often has one real direction per node at every frequency:
 * J~[k][q] = u_q s[k][q] (the literal linearly polarised, the radially and
 * the azimuthally polarised Gaussians with any spectral amplitude and phase;
 * not the curl-consistent linear beam, whose longitudinal magnetic term turns
 * n x B with k).  Then
 *   J~ g = u (s g)   and   (J~ h) x R = (s h)(u x R),
 * with u x R shared by the frequencies, so each (point, frequency, node)
 * term needs about a third fewer operations.  The library tests every node
 * of the FP64 tables once per table set (residual |J~ - u (u.J~)| against
 * max_k |J~|, u the unit direction of the largest J~ of the node).  When
 * every residual is below 1e-10, SC_FP32_SPLIT uses FP32 tables of
 * (s, rho~) per (k, node) (16 B) and node records of (x, y, z, |r_s|, u)
 * (32 B); when below 1e-14 (the built-in beams that factor do so to
 * rounding), SC_FP64 uses the same records in FP64 (32 B and 64 B, built
 * at the first FP64 evaluation); otherwise the general tables.  The sums
 * are the same up to rounding (the same tolerances against the oracle
 * apply); results are reproducible and independent of the launch shape
 * either way, and a batch may mix factored and general problems.
 *
 * Tied charge.  When moreover rho~[k][q] = -i beta_q s[k][q] / k with a real
 * beta_q per node (a factoring beam with no longitudinal field, B = -z x E:
 * the literal linear, radial and azimuthal Gaussians, Laguerre-Gauss sets
 * whose current factors; rho~ = (2W/4pi)(n.E) P and J~ = ik (2W/4pi)(n x B) P
 * then carry the same amplitude; not the curl-consistent radial beam, whose
 * E_z turns n.E by 90 degrees), the charge term needs no product of its
 * own: with A = s e^{ik delta} and m = ik - 1/R,
 *   rho~ (m e^{ik delta} / R^2) R = beta (R / R^2) (-i A m / k),
 * and the B term (A m) (u x R / R^2) keeps A m / k with the factor k applied
 * after the sum, so a (point, frequency, node) term takes about 30 % fewer
 * operations than with the factored current alone (26 vector instructions
 * against 37 in FP32, with s in polar form).  The same test
 * decides it (residual |rho~ + i beta s / k| against the node's largest
 * (|rho~|^2 + |J~ / k|^2)^1/2, same tolerances); rim nodes, which carry a
 * charge only, take u = 0, beta = 1 and s = i k rho~.  The tables are the
 * factored ones plus beta per node (4 B in FP32, 8 B in FP64) and, for
 * SC_FP32_SPLIT, s in polar form (|s|, arg s / 2pi), 8 B per (k, node),
 * whose phase joins the sine's argument.
 * enable = 1 (default) uses the factored tables whenever the test passes,
 * with the tied charge where it holds; 2 the factored current without the
 * tied charge; 0 neither.  The test needs the FP64 tables: with keep_fp64 = 0
 * it runs when the incident field is set, so enabling afterwards has no
 * effect until the field is set again.  SC_E_INVAL for another value.      */
sc_status sc_set_factoring(sc_prob *p, int enable);
/* *active = the table layout evaluation of p in precision prec uses: 0 the
 * general tables, 1 the factored current, 2 the factored current with the
 * tied charge (runs the test if it has not run yet; always 0 for SC_FP32).
 * SC_E_STATE without an incident field, SC_E_INVAL for an unknown precision. */
sc_status sc_get_factoring_for(sc_prob *p, sc_precision prec, int *active);
/* sc_get_factoring_for(p, SC_FP32_SPLIT, active).                          */
sc_status sc_get_factoring(sc_prob *p, int *active);

/* The observation points r' where the reflected field is evaluated (Sec.
 * III-C: the focal region, discretised separately from the mirror; the
 * paper's domain decomposition splits these points across processes, here
 * they are the tiles of one launch), [n_obs][3] doubles, n_obs >= 1 (host or
 * device per on_device); SC_E_INVAL for non-finite host points.  From host points the library also takes max |r'|, which lets
 * SC_FP32_SPLIT skip the fractional-turn reduction of the per-pair phase
 * (k_max |r'| / 2pi < 250 turns), and lets both split forms (SC_FP32_SPLIT
 * and SC_FP64) form delta = |r_s - r'| - |r_s| and 1/|r_s - r'| by short
 * series (when |r'| <= 4e-4 |r_s| on every node); the choice is per problem
 * and changes the rounding, not the tolerance.  Device points always take
 * the general forms.
 * Accuracy away from the focus: SC_FP32_SPLIT rounds the per-pair phase
 * k delta (|k delta| <= k |r'|) to FP32, an error of about k |r'| 2^-24 rad
 * per term (1e-4 rad at |r'| = 300 wavelengths), so its relative error grows
 * linearly with the distance of the points from the focus; SC_FP64 holds
 * about k |r'| 2^-53 rad.                                                   */
sc_status sc_set_observation(sc_prob *p, const double *xyz, int n_obs, int on_device);

/* Evaluate the reflected spectral field at every (observation point, k): the
 * Stokes-converted physical-optics integrals of Sec. II (eq.
 * stratton-chu-poa-og, with the rim line integral) by the mirror's quadrature,
 * in the arithmetic `prec` (see sc_precision).
 * E, B: [n_k][n_obs][3] complex128 (SC_FP64) or complex64 (FP32 forms),
 * host or device per on_device; either may be NULL to keep the result only
 * on the device (for sc_to_time / sc_to_time_at / sc_get_result).  Needs mirror, frequencies,
 * incident field and observation points (SC_E_STATE).                      */
sc_status sc_evaluate(sc_prob *p, sc_precision prec, void *E, void *B, int on_device);
/* sc_evaluate for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the call allocates
 * nothing, device or host.  Its scratch memory (work counters, the job
 * record, the split-K partials) is a static device array of
 * SC_NOALLOC_SCRATCH_BYTES on each GPU, which the library holds until the
 * process ends.
 * E, B: DEVICE arrays [n_k][n_obs][3] of complex128 (SC_FP64) or complex64
 * (the FP32 forms), written by the stream work enqueued here.  Requires the
 * problem's tables of `prec` to be built (SC_E_STATE otherwise): one
 * sc_evaluate of the problem in that precision since its mirror, frequencies
 * or incident field last changed builds them (the FP32-split tables of a
 * field whose current factors are built when the field is set).  Its split-K
 * partials, 12 x
 * ceil(nodes / chunk) x n_k x n_obs (padded to 128) reals of the precision,
 * must fit in SC_NOALLOC_SCRATCH_BYTES - 1024 bytes (SC_E_INVAL otherwise).
 * The results equal sc_evaluate's bit for bit with the same launch shape; the
 * problem's stored result (sc_get_result, sc_to_time*) is left as it was.
 * Every call on a GPU shares that GPU's array and leaves its contents there
 * (each call clears the counters it needs): calls that overlap on one GPU,
 * from other streams, contexts or threads, race and give wrong results.     */
#define SC_NOALLOC_SCRATCH_BYTES (64u << 20)
sc_status sc_evaluate_noalloc(sc_prob *p, sc_precision prec, void *E, void *B);

/* Copy the last result (same layout and type as sc_evaluate).              */
sc_status sc_get_result(const sc_prob *p, void *E, void *B, int on_device);

/* Semi-discrete transform of the last result to time (Sec. III-B,
 * eq. impl.semiDiscreteFFT, the sum over the positive-frequency samples):
 *   F(t_m) = dk * sum_n F_n e^{-i k_n t_m}
 * (complex; the physical field is 2 Re F(t)), at the n_t <= SC_MAX_TIMES
 * uniform times t_m = t0 + m dt, with dk the step of the problem's uniformly
 * spaced frequencies (at least two, spaced to 1e-12 relative; SC_E_INVAL
 * otherwise).  Et, Bt: [n_t][n_obs][3], the complex type of the result, host
 * or device per on_device (either may be NULL to keep them on the device).
 * SC_E_STATE without a result.                                              */
sc_status sc_to_time(sc_prob *p, double t0, double dt, int n_t, void *Et, void *Bt, int on_device);
/* The same sum at arbitrary times t[n_t] (host array) with the weight dk given
 * (any frequency grid, e.g. the trapezoid or quadrature weight of a
 * non-uniform one).                                                         */
sc_status sc_to_time_at(sc_prob *p, double dk, const double *t, int n_t, void *Et, void *Bt, int on_device);

/* ------------------------------------------------------------ diagnostics */
/* Verification of the reflected field as in Sec. IV-A: Maxwell residuals in
 * the frequency and time domains and the energy in the observation volume.
 * The residuals use 4th-order central differences on a 13-point stencil per
 * point: the point itself, then offsets -2h, -h, +h, +2h along x, then along
 * y, then along z.  Workflow: sc_stencil_points -> sc_set_observation with
 * the 13 n_pts stencil points -> sc_evaluate (any precision) -> the calls
 * below, which read the problem's last result.                              */

/* Host helper: out [n_pts * 13][3] = the stencil of each point of xyz [n_pts][3]. */
sc_status sc_stencil_points(const double *xyz, int n_pts, double h, double *out);
/* Frequency-domain residual (eq. relDiffMaxwellFreq), for every k and point:
 *   e_f = 2 (curl E - ik B) / (max|curl E| + max|ik B|)
 *       + 2 (curl B + ik E) / (max|curl B| + max|ik E|),
 * maxima over the n_pts points at the same k; ef [n_k][n_pts] (host) = |e_f|.
 * SC_E_STATE without a result, or if the observation set is not 13 n_pts.   */
sc_status sc_maxwell_residual_freq(sc_prob *p, int n_pts, double h, double *ef);
/* Time-domain residual (eq. relDiffMaxwellTime) at times t [n_t] (host), on
 * the physical fields 2 Re F(t), F(t) = dk sum_n F_n e^{-i k_n t}:
 *   e_t = 2 (curl E + dB/dt) / (max|curl E| + max|dB/dt|)
 *       + 2 (curl B - dE/dt) / (max|curl B| + max|dE/dt|),
 * time derivatives by 4th-order central differences of step dt;
 * et [n_t][n_pts] (host) = |e_t|; n_t <= SC_MAX_TIMES / 5.                   */
sc_status sc_maxwell_residual_time(sc_prob *p, int n_pts, double h, const double *t, int n_t, double dt,
                                   double dk, double *et);
/* Electromagnetic energy of the observation set at times t [n_t] (host), each
 * point standing for a cell of volume dV (Lorentz-Heaviside, c = 1, Sec. IV-A):
 *   W(t) = 1/2 dV sum_points ( |2 Re E(t)|^2 + |2 Re B(t)|^2 ).
 * W [n_t] (host), n_t <= SC_MAX_FREQUENCIES.  Reads the last result; any
 * observation set.                                                          */
sc_status sc_field_energy(sc_prob *p, const double *t, int n_t, double dk, double dV, double *W);

/* Evaluate several problems in ONE persistent launch (tiles of all problems
 * share the device), then reduce each; results are kept per problem (read
 * with sc_get_result).  The launch shape is the context's batch launch
 * (sc_set_batch_launch, sc_autotune_batch) or the library's.  The split-K
 * partials of the batch (12 reals per chunk, frequency and point of each
 * problem) are kept within max(2 x 16 B x sum of frequencies x nodes, 8 GiB),
 * doubled for SC_FP64: if the chunks so far exceed that, the problems that fix
 * no chunk with sc_set_launch take the smallest power-of-two chunk from 2048
 * up that fits (sc_get_timing reports each problem's chunk).  Each problem's
 * result is bitwise identical to what sc_evaluate gives it alone with the
 * same chunk.                                                               */
sc_status sc_evaluate_batch(sc_ctx *ctx, sc_prob *const *probs, int n, sc_precision prec);

/* Device bytes held by the problem (tables, observation data, results).    */
sc_status sc_prob_device_bytes(const sc_prob *p, size_t *bytes);

/* ------------------------------------------------------------------ serving */

/* A field-solve request (all arrays are host memory, copied at submit). */
typedef struct {
    double f, r_max;          /* mirror                                       */
    int n_r, n_phi;           /* quadrature                                   */
    int n_k;                  /* frequencies                                  */
    const double *k;          /* [n_k]                                        */
    const double *spectrum;   /* complex128 [n_k] or NULL                     */
    double w0, pol_angle;     /* beam waist and polarisation (see below)      */
    int consistent;           /* beam variant, see sc_set_incident_beam       */
    int n_obs;                /* observation points                           */
    const double *obs;        /* [n_obs][3]                                   */
    sc_precision prec;        /* arithmetic                                   */
    int n_t;                  /* 0, or number of time samples                 */
    const double *t;          /* [n_t] time samples                           */
    double dk;                /* transform weight                             */
    int beam;                 /* sc_beam of the incident field                */
} sc_request;

typedef struct {
    double queue_ms;          /* submit -> admitted                           */
    double run_ms;            /* admitted -> result ready on host             */
    double total_ms;          /* submit -> result ready                       */
    int64_t evals;            /* obs x freq x surface nodes                   */
    size_t device_bytes;      /* HBM charged against the budget: the set-up's
                                 peak at admission, what the prepared request
                                 holds once its tables are built              */
} sc_request_stats;

typedef struct {
    int64_t submitted, admitted, completed, rejected, cancelled, queued, running;
    size_t hbm_in_use, hbm_budget;
    int64_t launches;         /* scheduling quanta launched                    */
    int64_t evals_done;       /* evaluations of completed requests            */
    int64_t evals_launched;   /* evaluations in the launched quanta           */
    double quad_ms;           /* device time of the completed quanta (events) */
    double prep_ms;           /* summed per request: start of its set-up to its
                                 tables ready (includes waiting for the device) */
    double prep_host_ms;      /* host time of the preparation thread's set-up
                                 calls (no waiting)                           */
    size_t host_in_use, host_budget;   /* pinned host bytes of admitted requests
                                 whose results are not yet collected, and
                                 their limit (a quarter of the host memory, at
                                 most 64 GiB): admission waits for collection */
} sc_server_stats;

/* Start a serving loop on `ctx`: requests are admitted while their HBM
 * footprint fits `hbm_budget` bytes and at most `max_running` are in flight;
 * the tiles of all admitted requests are scheduled together in persistent
 * launches of about `quantum_ms` of work, so requests that arrive while
 * others run join the next launch (continuous batching).  The server owns a
 * host thread and uses `ctx` exclusively until destroyed.                  */
sc_status sc_server_create(sc_ctx *ctx, size_t hbm_budget, int max_running, double quantum_ms,
                           sc_server **out);
/* Queue a request; returns a ticket.  SC_E_REJECTED if it can never fit.   */
sc_status sc_server_submit(sc_server *s, const sc_request *req, uint64_t *ticket);
/* Wait up to timeout_ms (< 0: forever) for a result.  E, B: host arrays
 * [n_k][n_obs][3] (complex128 for SC_FP64, complex64 otherwise); Et, Bt:
 * [n_t][n_obs][3] or NULL.  The ticket is released unless the wait timed
 * out (SC_E_TIMEOUT).  Any number of threads may wait on different tickets;
 * all waits must have returned before sc_server_destroy.                   */
sc_status sc_server_wait(sc_server *s, uint64_t ticket, double timeout_ms, void *E, void *B,
                         void *Et, void *Bt, sc_request_stats *stats);
/* Cancel a queued request (running requests finish normally).              */
sc_status sc_server_cancel(sc_server *s, uint64_t ticket);
sc_status sc_server_get_stats(sc_server *s, sc_server_stats *out);
/* Stop the loop after in-flight work completes and free everything.        */
sc_status sc_server_destroy(sc_server *s);

#ifdef __cplusplus
}
#endif

#endif /* SC_H */
