/*
 * qed.h - C ABI of the MI355X (gfx950) QED Monte Carlo particle step.
 *
 * Method: Wang, Sheng, Gibbon & Li, "Modeling of photon and pair production due
 * to quantum electrodynamics effects in particle-in-cell simulation",
 * arXiv:1608.06356.  Photon emission (nonlinear Compton) with the spectrum of
 * Eq. (1) ("formula I") or Eq. (4) ("formula II"), pair creation (Breit-Wheeler)
 * with Eq. (6), quantum parameters chi_e / chi_ph from Eqs. (2)-(3), photon
 * energies by inverting the cumulative spectrum (Eq. 7) with the infrared cutoff
 * xi_min eps_e = 2 m_e c^2, and the event generator of the paper's method II
 * written as an optical depth.
 *
 * Units (the paper's normalisation, stated below Eqs. 2-3): time 1/omega_0,
 * length c/omega_0, momentum m_e c, fields m_e c omega_0 / e.  The Schwinger field
 * is E_S = m_e c^2 / (hbar omega_0) at lambda_0 = 1 um (412148.4...).
 *
 * Conventions for every entry point
 *   - Return QED_OK (0) or a negative QED_ERR_* code; qed_last_error() gives text.
 *   - Argument errors are detected on the host before anything is enqueued.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 *     asynchronous.  Device-side conditions (capacity exceeded, NaN chi, chi out of
 *     table range, scan time-out) set counters in the context; qed_get_status()
 *     synchronises the stream and returns and clears them.
 *   - Every particle and field buffer is device memory owned by the caller, which
 *     must keep it alive until the enqueued work has finished.  The library only
 *     allocates its own context memory (tables, emitter list, counters, scan state)
 *     in qed_create / qed_build_tables / qed_reserve, or on the first use of a
 *     larger species (see qed_reserve).
 *   - Particle counts live in device memory (qed_species_t.count), so a sequence of
 *     calls needs no host synchronisation.
 *
 * Ordering contract: appended particles are ordered by (parent index, event
 * number); new ids are next_id + rank (photons) or next_id + 2 rank and
 * next_id + 2 rank + 1 (electron, positron of pair `rank`).  Given identical
 * decisions, counts and positions of every appended or compacted particle are
 * deterministic and independent of the launch configuration.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (id_lo, id_hi ^ seed),
 * counter = (step_lo, (step_hi & 0xFFFFFF) | purpose << 24, k, 0); uniform
 * u = ((x >> 9) + 0.5) * 2^-23.
 */
#ifndef QED_H
#define QED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define QED_OK            0
#define QED_ERR_ARG      (-1)   /* invalid argument (null pointer, size, enum)   */
#define QED_ERR_HIP      (-2)   /* a HIP runtime call failed                     */
#define QED_ERR_CAPACITY (-3)   /* an append exceeded a species' capacity        */
#define QED_ERR_RANGE    (-4)   /* a size beyond what the context was reserved for */
#define QED_ERR_STATE    (-5)   /* call order violated (tables missing, ...)     */

/* element type of positions and momenta */
#define QED_F32 0
#define QED_F64 1

/* photon spectrum used for the emission tables */
/* qed_sample: table copy, or the surrogate networks with table fallback */
#define QED_SAMPLER_MLP 2

#define QED_FORMULA_I  1        /* Eq. (1) */
#define QED_FORMULA_II 2        /* Eq. (4) */
#define QED_FORMULA_CLASSICAL 3 /* Eq. (5), the hbar -> 0 limit, with z = 2 xi / (3 chi),
                                   restricted to xi < 1 like the quantum spectra */

/* field kinds */
#define QED_FIELD_UNIFORM      0   /* E, B constant (qed_fields_t.E/B)             */
#define QED_FIELD_GRID         1   /* periodic collocated grid, quadratic (TSC)    */
#define QED_FIELD_PER_PARTICLE 2   /* one E, B per particle (arrays indexed like x) */

/* qed_params_t.flags */
#define QED_FLAG_NO_RECOIL     1u  /* leptons keep their momentum when emitting   */
#define QED_FLAG_STATIC_PHOTONS 2u /* qed_create_pairs does not move photons      */
#define QED_FLAG_TRACK_DEAD    4u  /* only qed_create_pairs kills particles: lets
                                      qed_compact skip when nothing died (below)   */
#define QED_FLAG_SURROGATE     8u  /* float32 species: rates and xi from the trained
                                      surrogate nets (table fallback), see below   */
#define QED_FLAG_METHOD_I     16u  /* the paper's method I generator (text after
                                      Eq. 7): an event in a (sub-)step if W Dt > r_1,
                                      at most one per sub-step, with the step split
                                      into N = ceil(W Dt / 0.2) sub-steps             */
#define QED_FLAG_NO_SUBSTEP   32u  /* with QED_FLAG_METHOD_I: N = 1 (no adaptive step) */

#define QED_DEAD_ID UINT64_MAX     /* id of a particle removed by pair creation */
#define QED_STEP_DEVICE (-1)       /* step argument: use the context's device step index */

#if defined(__GNUC__)
#define QED_API __attribute__((visibility("default")))
#else
#define QED_API
#endif

typedef struct qed_ctx *qed_ctx_t;

typedef struct {
  uint32_t seed;      /* xor-ed into the Philox key                                  */
  int32_t  kmax;      /* max events per lepton per step, 1..8 (cap is counted)       */
  uint32_t flags;     /* QED_FLAG_*                                                  */
  int32_t  reserved;
} qed_params_t;

/* Structure-of-arrays particle storage (caller-owned device memory).
   Leptons: p = momentum.  Photons: p = k = gamma_ph * direction.
   Live particles are [0, *count); each array holds `capacity` elements. */
typedef struct {
  int32_t   dtype;             /* QED_F32 or QED_F64: type of x..pz        */
  int32_t   reserved;
  void     *x, *y, *z;
  void     *px, *py, *pz;
  double   *tau;               /* optical depth (always float64)            */
  uint64_t *id;                /* unique id; QED_DEAD_ID marks a dead one   */
  int64_t   capacity;
  int64_t  *count;             /* device int64                              */
} qed_species_t;

typedef struct {
  int32_t kind;                /* QED_FIELD_*                                          */
  int32_t nx, ny, nz;          /* GRID: nodes per axis                                 */
  const float *grid;           /* GRID: 6 floats per node (Ex Ey Ez Bx By Bz),
                                  node (i,j,k) at ((k*ny + j)*nx + i)*6; node i sits at
                                  x = i*dx; the box [0, n*d) is periodic; at most
                                  2^32 - 1 floats (nx*ny*nz*6), QED_ERR_ARG beyond   */
  double dx, dy, dz;
  double E[3], B[3];           /* UNIFORM                                              */
  const float *pE[3], *pB[3];  /* PER_PARTICLE: device arrays, element i for particle i */
} qed_fields_t;

/* Device-side event counters, accumulated since the last qed_get_status. */
typedef struct {
  int64_t events;              /* lepton optical-depth events                 */
  int64_t photons;             /* photons appended                            */
  int64_t rejected;            /* events below xi_min = 2/gamma (thinned)     */
  int64_t capped;              /* leptons that reached kmax events in a step  */
  int64_t pairs;               /* pairs appended                              */
  int64_t dropped;             /* appends lost to a full species              */
  int64_t chi_out_of_range;    /* lookups outside the tables' chi range        */
  int64_t nan_chi;             /* particles skipped because chi was not finite */
  int64_t scan_timeouts;       /* prefix-scan waits that gave up (must be 0)  */
  int64_t compacted;           /* particles removed by qed_compact            */
  int64_t mlp_fallback_xi;     /* surrogate xi samples that fell back to the table */
  int64_t mlp_fallback_rate;   /* surrogate rates that fell back to the table     */
  int64_t thinned;             /* surrogate path: candidate events not kept (thinning) */
  int64_t envelope_exceeded;   /* surrogate path: a rate outside [0.89, 1] x its envelope (must be 0) */
  int64_t retired;             /* photons retired into the tally (qed_set_retirement) */
  int64_t box_fallback;        /* lepton-pass workgroups on a grid whose stencil box did
                                  not fit in LDS (they gather from global memory: a
                                  sign that the species needs qed_sort_by_cell) */
} qed_counters_t;

/* Surrogate training (not part of the paper; see qed_surrogate_train). */
typedef struct {
  int64_t steps;       /* Adam steps per net                                     */
  int64_t batch;       /* samples per step (drawn from the float64 master tables) */
  double lr;           /* peak learning rate (cosine decay to 0)                  */
  uint32_t seed;
  int32_t nets;        /* bit 0: xi net (A), bit 1: rate net (B)                  */
} qed_train_spec_t;

/* Creates a context on the current HIP device.  Allocates counters only. */
QED_API int qed_create(qed_ctx_t *ctx, const qed_params_t *params);
QED_API void qed_destroy(qed_ctx_t ctx);
QED_API const char *qed_last_error(qed_ctx_t ctx);

/* Reserves the context's scan state for species of up to `max_particles`
   elements and its emitter list (one 128-byte record slot, one mask bit and one
   list entry per lepton) for lepton species of up to `max_particles` (allocates;
   call before graph capture).  Without it, or when a species is larger, the
   entry points grow what they need on first use: the scan state in every entry
   point that appends or compacts, the emitter list in qed_gather_push for the
   leptons passed to it, so a large photon species costs no emitter slots.  Such
   a growing first use synchronises the device and must not be under capture. */
QED_API int qed_reserve(qed_ctx_t ctx, int64_t max_particles);

/* Sets the next id handed to appended particles (device counter). */
QED_API int qed_set_next_id(qed_ctx_t ctx, uint64_t next_id, void *stream);
QED_API int qed_get_next_id(qed_ctx_t ctx, uint64_t *next_id, void *stream);   /* syncs */

/* Builds all tables on the device in float64 by quadrature of the paper's spectra:
   the photon rate h(chi) and inverse CDF (Eq. 1 if formula == QED_FORMULA_I,
   Eq. 4 if QED_FORMULA_II, Eq. 5 if QED_FORMULA_CLASSICAL; text after Eq. 7) on 256 chi nodes over [1e-3, 1e2],
   256 quantile nodes each; the pair rate (Eq. 6) on 512 chi nodes over [1e-2, 1e2]
   and the half-spectrum inverse CDF on 256 x 256 nodes.  Also writes the float32 /
   16-bit copies the single-precision kernels stage in LDS. */
QED_API int qed_build_tables(qed_ctx_t ctx, int formula, void *stream);

/* Same as qed_build_tables with the upper ends of the chi ranges chosen by the
   caller: photon tables on 256 log nodes over [1e-3, rad_chi_max], pair tables
   over [1e-2, pair_chi_max] (same node counts).  Needed where chi exceeds 1e2, as
   for the single electron of chi_0 ~ 4e4 in the cascade of Fig. 5; the node
   spacing grows with the range.  Requires 1 <= rad_chi_max <= 1e6 and
   10 <= pair_chi_max <= 1e6 (QED_ERR_ARG otherwise).  The surrogate nets cover
   chi in [1e-3, 1e2] only: with any other range the surrogate entry points and
   QED_FLAG_SURROGATE return QED_ERR_STATE. */
QED_API int qed_build_tables_range(qed_ctx_t ctx, int formula, double rad_chi_max, double pair_chi_max,
                                   void *stream);

/* Copies a table to host memory (synchronous).  which: 0 rad ln h [256] f64,
   1 rad logit-xi quantiles [256*256] f64, 2 pair ln h + 8/(3 chi) [512] f64,
   3 pair quantiles [256*256] f64, 4 rad 16-bit codes [256*256] u16,
   5 rad row offset/scale [2*256] f32, 6 pair 16-bit codes, 7 pair offset/scale. */
QED_API int qed_get_table(qed_ctx_t ctx, int which, void *host, size_t bytes);

/* tau = -ln u for particles [0, *count) (Philox purpose 0, counter k = 0). */
QED_API int qed_init_optical_depth(qed_ctx_t ctx, qed_species_t *sp, int64_t step, void *stream);

/* Fills a grid with the circularly polarised standing wave
   E = a0 cos x (0, cos t, sin t), B = a0 sin x (0, cos t, sin t) at time t on n^3
   nodes of spacing L/n (layout of qed_fields_t.grid). */
QED_API int qed_fill_standing_wave(qed_ctx_t ctx, float *grid, int n, double L, double a0,
                           double t, void *stream);

/* Step index in device memory, so that one captured hipGraph of a step can be
   replayed: pass step = QED_STEP_DEVICE to the entry points that take a step
   (their random streams then use the device index), fill the grid with
   qed_fill_standing_wave_at_step (t = t0 + dt * step), and end the step with
   qed_advance_step.  All three enqueue small kernels only (no memset, no host
   synchronisation). */
QED_API int qed_set_step(qed_ctx_t ctx, int64_t step, void *stream);
QED_API int qed_advance_step(qed_ctx_t ctx, void *stream);
QED_API int qed_fill_standing_wave_at_step(qed_ctx_t ctx, float *grid, int n, double L, double a0,
                                           double t0, double dt, void *stream);

/* Lepton pass, every particle [0, *count): field at x^n, relativistic Boris push
   (charge = -1 electron, +1 positron), x^{n+1} = x^n + v dt (wrapped into a GRID
   box), chi_e from Eq. (2) in float64, W = alpha E_S h(chi)/gamma, and the optical
   depth decrement tau -= W dt.  Particles whose optical depth runs out within the
   step are flagged in the context's emitter mask (one bit per particle) and their
   record (fields seen, chi, W, time left after the first event) is kept at their
   index; qed_emit_photons lists them in index order and finishes them.  One kernel
   launch: two particles per thread for a float32 species on a GRID whose capacity
   is at least 64 particles per cell, one otherwise (the two agree to float32
   rounding).  With QED_FLAG_SURROGATE (float32) the optical depth runs down at a
   closed-form envelope of the rate evaluated at a float32 upper bound of chi
   (Poisson thinning: qed_emit_photons evaluates chi in float64 and keeps each
   candidate event with probability W / W_env).  Fails with QED_ERR_STATE if the
   tables are missing. */
QED_API int qed_gather_push(qed_ctx_t ctx, const qed_fields_t *fields, qed_species_t *leptons,
                    int charge, double dt, int64_t step, void *stream);

/* Emission events of the emitters found by the last qed_gather_push on `leptons`:
   per event k draws xi from the inverse CDF (Eq. 7), rejects xi < 2/gamma, appends
   a photon of energy xi gamma along p with its own optical depth, recoils the lepton
   to (1 - xi) gamma, draws a new tau, and continues while the optical depth runs out
   again within the step (at most kmax events).  Photons are appended after
   photons->count in (emitter index, k) order; with QED_FLAG_SURROGATE (float32)
   the first events of all emitters come first, in emitter order, then the later
   events of the emitters that have them, in (emitter index, k) order. */
QED_API int qed_emit_photons(qed_ctx_t ctx, qed_species_t *leptons, qed_species_t *photons,
                     int64_t step, void *stream);

/* Photon pass, every photon [0, *count): ballistic move (unless
   QED_FLAG_STATIC_PHOTONS), chi_ph from Eq. (3), W_pair = alpha E_S h_pair/gamma_ph
   (zero below gamma_ph = 2), optical depth; on an event xi = eps_e/eps_ph from the
   half-spectrum of Eq. (6), the electron gets xi gamma_ph and the positron the rest,
   both along the photon, appended at the same rank; the photon's id becomes
   QED_DEAD_ID (remove it with qed_compact).  Pairs are ranked in photon order.
   Float32 species: a streaming launch takes every photon's step and marks the
   photons with an event in a ballot mask, a second lists them in photon order
   and a third makes their pairs (then a one-thread launch advances the counts);
   float64 species: one launch.  With QED_FLAG_SURROGATE (float32) the optical
   depth runs down at the envelope alpha E_S h_pair_env(chi_ph) / gamma_ph, or,
   after qed_set_retirement, at the largest pair rate W_max(gamma_ph) the field
   bound allows (no field gathered), and each candidate event is kept with
   probability W / W_env, W from the pair head of the rate net (Poisson
   thinning; the table where the net's output fails its check).  The event mask
   and list are sized for the photon capacity on the first call with a larger
   capacity (allocation: not under graph capture). */
QED_API int qed_create_pairs(qed_ctx_t ctx, const qed_fields_t *fields, qed_species_t *photons,
                     qed_species_t *electrons, qed_species_t *positrons, double dt,
                     int64_t step, void *stream);

/* Stable reordering of src into dst (caller-owned, same dtype, capacity >= src's)
   by the grid cell of each particle's nearest node, so that the quadratic-spline
   gather of neighbouring threads reads neighbouring nodes.  Key of node (i,j,k):
   cells grouped in 4x4x4 blocks, blocks along the Morton curve of their
   coordinates (i/4, j/4, k/4) (bit b of i/4, j/4, k/4 to bits 3b, 3b+1, 3b+2) and
   cells in z-major order inside a block: Morton(i/4, j/4, k/4) * 64 +
   ((k%4) * 4 + j%4) * 4 + i%4.  Grids with more than 256 blocks along an axis
   (3 bits per block-coordinate bit would overflow the 32-bit key) order the
   blocks z-major instead: ((k/4 * NBy + j/4) * NBx + i/4), NBx = ceil(nx/4),
   NBy = ceil(ny/4).  Ids, optical depths
   and therefore every random stream move with the particles.  A periodic sort is
   what keeps qed_gather_push's field reads local.  Sorts the *count particles
   present: reads the count from the device, which synchronises `stream`.
   Allocates its scratch on the first call for a given capacity; not for graph
   capture. */
QED_API int qed_sort_by_cell(qed_ctx_t ctx, const qed_fields_t *fields, qed_species_t *src,
                             qed_species_t *dst, void *stream);

/* Stable in-place removal of particles whose id is QED_DEAD_ID.  With
   QED_FLAG_TRACK_DEAD the context remembers the species it compacted last;
   qed_create_pairs on that species counts the photons it kills, and a later
   qed_compact with nothing killed returns at once on the device (no host
   synchronisation).  Without the flag every call scans the whole species. */
QED_API int qed_compact(qed_ctx_t ctx, qed_species_t *sp, void *stream);

/* qed_compact with no allocation, for callers that cannot allocate device
   memory (code under graph capture, serving loops, harnesses that forbid
   hipMalloc).  Same result as qed_compact (same kernels, same QED_FLAG_TRACK_DEAD
   behaviour); the scan state lives in a static device array of the library
   (513 KiB per GPU, held until the process ends) instead of context memory, so
   species are limited to capacity <= 2^26 (QED_ERR_RANGE beyond, detected on
   the host before anything is enqueued).  Every call on one GPU shares that
   array and clears it at its start: calls that overlap on one GPU (other
   streams, other contexts, other threads) race and must be ordered by the
   caller. */
QED_API int qed_compact_static(qed_ctx_t ctx, qed_species_t *sp, void *stream);

/* Photon retirement, for runs whose photon population outgrows memory.  Pair
   creation can only take a photon's optical depth tau to zero at the pair rate
   W = alpha E_S h_pair(chi_ph) / gamma_ph (Eq. 6), and chi_ph = gamma_ph / E_S
   |k x (E + k x B)| <= gamma_ph F / E_S if F bounds |E| + |B| for the rest of the
   run.  With the caller's end time t_end (t = step dt) and bound F, a photon whose
   tau exceeds W_max (t_end - t), W_max the pair-rate envelope at that chi bound,
   cannot convert before t_end: qed_emit_photons does not store such a new photon
   and qed_create_pairs marks such a photon dead (QED_DEAD_ID, removed by
   qed_compact); either way its gamma_ph is counted into the tally, a histogram of
   QED_TALLY_BINS bins uniform in ln gamma_ph over [ln 2, ln 1e7]
   (bin = floor((ln gamma - ln 2) / ((ln 1e7 - ln 2) / QED_TALLY_BINS)), clamped).
   Ids still count every emitted photon, so the stored photons keep the ids and
   random streams they would have without retirement, and no pair changes.
   t_end = 0 switches retirement off.  The first call allocates the tally (not
   under graph capture).  qed_tally_species adds the live photons of a species
   (id != QED_DEAD_ID, gamma_ph = |k|) to the tally; qed_get_tally synchronises
   `stream`, copies the QED_TALLY_BINS counts to host memory and clears them if
   `clear`.  Both need the tally (QED_ERR_STATE before qed_set_retirement). */
#define QED_TALLY_BINS 65536
QED_API int qed_set_retirement(qed_ctx_t ctx, double t_end, double field_bound);
QED_API int qed_tally_species(qed_ctx_t ctx, const qed_species_t *photons, void *stream);
QED_API int qed_get_tally(qed_ctx_t ctx, uint64_t *host_counts, int64_t nbins, int clear, void *stream);

/* Quantum parameter of every particle [0, *count) of a species at its current
   momentum and the fields at its position (uniform, grid or per-particle, as in
   the step): kind QED_CHI_LEPTON evaluates Eq. (2) with v = p / gamma,
   QED_CHI_PHOTON Eq. (3) with |v| = 1 and gamma_ph = |k|.  The same device code
   as the step: float64 arithmetic throughout (float32 species: on the float32
   values, which float64 holds exactly), in the rearranged form that avoids the
   cancellation of (E + v x B)^2 - (v . E)^2 for ultra-relativistic particles.
   Writes chi[i] (device float64 array of at least *count elements). */
#define QED_CHI_LEPTON 0
#define QED_CHI_PHOTON 1
QED_API int qed_eval_chi(qed_ctx_t ctx, const qed_fields_t *fields, const qed_species_t *sp, int kind,
                         double *chi, void *stream);

/* Standalone lookups: for n particles with chi (f64) and gamma (f64) and the ids
   used for their streams, writes ln W_rad (f32, uncut rate, -inf if zero) and one
   xi sample (f32, event k = 0 of `step`); precision selects the table copy:
   QED_F64 master tables or QED_F32 (16-bit LDS copy).  ln W_pair likewise if
   lnw_pair != NULL (gamma taken as gamma_ph). */
QED_API int qed_sample(qed_ctx_t ctx, const double *chi, const double *gamma, const uint64_t *id,
               int64_t n, int precision, int64_t step, float *lnw_rad, float *xi,
               float *lnw_pair, void *stream);

/* Surrogate networks.  Not in the paper: two multilayer perceptrons (3 hidden
   layers of 64, SiLU) replace table lookups, the tables staying the fallback.
   Net A (0): (log10 chi, logit u) -> logit(xi) - ln chi - 3 ln u; net B (1):
   log10 chi -> (ln h_rad - ln chi, ln h_pair + 8/(3 chi) - ln chi), with fixed
   affine normalisations.  The 64x64 layers run on BF16 matrix cores with a two-term
   split of every operand (three products, float32 accumulation).
   qed_surrogate_train: trains the nets selected by spec->nets with Adam on batches
   drawn (Philox, spec->seed) from the float64 master tables; requires
   qed_build_tables.  qed_surrogate_params: parameter count of a net.
   qed_surrogate_io: copies a net's float32 parameters to (direction 0) or from
   (direction 1) host memory; layout W1 b1 W2 b2 W3 b3 W4 b4 (row-major [out][in]).
   qed_surrogate_forward: raw normalised outputs for n inputs (device, [n][nin] ->
   [n][nout] float32), evaluated as the inference kernels evaluate it.  qed_surrogate_grad: gradient of the mean squared error
   sum_o mask*(y - t)^2 / n over an external batch (device float32 arrays) into
   grad (device, params floats).
   qed_sample with precision QED_SAMPLER_MLP uses both nets; a rate outside
   0 < h <= 1.001 * 5 chi / (2 sqrt3) or chi outside [1e-3, 1e2] falls back to the
   table, and a xi sample falls back when u is outside [1e-4, 1 - 1e-4] or the
   tabulated CDF at the predicted xi differs from u by more than 2e-3.  Fallbacks
   are counted (mlp_fallback_*).
   With QED_FLAG_SURROGATE in the context parameters, qed_gather_push,
   qed_emit_photons and qed_create_pairs on float32 species use the same nets and
   checks in place of the table lookups, through Poisson thinning.  The surrogate paths need both nets, trained or loaded
   (QED_ERR_STATE otherwise). */
QED_API int qed_surrogate_params(int net);
QED_API int qed_surrogate_train(qed_ctx_t ctx, const qed_train_spec_t *spec, void *stream);
QED_API int qed_surrogate_io(qed_ctx_t ctx, int net, float *host, size_t bytes, int direction);
QED_API int qed_surrogate_forward(qed_ctx_t ctx, int net, const float *x, int64_t n, float *y, void *stream);
QED_API int qed_surrogate_grad(qed_ctx_t ctx, int net, const float *x, const float *t, const float *mask,
                               int64_t n, float *grad, void *stream);

/* Synchronises `stream`, returns the counters and clears them.  Returns
   QED_ERR_CAPACITY if appends were dropped since the last call. */
QED_API int qed_get_status(qed_ctx_t ctx, qed_counters_t *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QED_H */
