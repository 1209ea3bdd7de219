/*
 * mclbm.h -- C ABI of the MI355X (gfx950) multi-component Shan-Chen lattice
 * Boltzmann solver with a coupled reactive advection-diffusion solute
 * (CooLBM method, arXiv 2502.12955).
 *
 * One time step, for every fluid node and every component s, performs the
 * paper's collide-stream update with inter-component forcing:
 *   - component densities and pseudo-potentials      eq:1.7, eq:1.11 /
 *                                                    pseudo-potential_multicomponent
 *   - cohesion force between components              eq:1.14
 *   - fluid-solid adhesion force                     eq:1.15
 *   - external body force rho_s * accel, added to the interaction force
 *     (Rayleigh-Taylor subsection)
 *   - Guo forcing (eq:1.19-1.21) or the Shan-Chen velocity shift (eq:1.17-1.18)
 *   - BGK collision with forcing term                eq:1.16, equilibrium eq:6
 *   - streaming with halfway bounce-back at solids and periodic wrap  eq:5
 * and for the solute (one reactive species):
 *   - ADE-BGK collision and streaming                eq:therpop_species,
 *                                                    eq:therpopeq_species
 *   - Kang wet-node first-order wall reaction, one missing link at a time
 *                                                    eq:wetnode9, eq:reactO2
 *   - optional inlet C = C_in at x = 0 and zero-gradient outlet at x = nx-1.
 *
 * Conventions for every host array exchanged through this ABI:
 *   node index n = x + nx * (y + ny * z), x fastest; N = nx * ny * nz.
 *   Field arrays are FP64 [field][N].  Solid nodes read as 0 on output.
 * Lattices: D2Q9 flow + D2Q5 solute (nz must be 1), or D3Q19 flow + D3Q7
 * solute.  Velocity order is that of the paper's tables; D3Q7 uses the first
 * seven D3Q19 vectors, D2Q5 the first five D2Q9 vectors.  Solute weights:
 * rest J0, links (1 - J0)/6 (3-D) or (1 - J0)/4 (2-D); solute c_s^2 =
 * (1 - J0)/3 or (1 - J0)/2; tau_d = D / c_s^2 + 1/2.
 *
 * Status codes: every int-returning call returns MCLBM_OK (0) or a negative
 * MCLBM_E* code; mclbm_last_error() gives the message of the last failure on
 * that handle.  All work is queued on the HIP stream given at init; calls
 * that return data to the host synchronise that stream.  A handle is not
 * thread-safe: use one handle per host thread.
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mclbm_handle mclbm_handle; /* opaque; owned by the library */

enum {
    MCLBM_OK = 0,
    MCLBM_EINVAL = -1,    /* bad parameter, size or layout */
    MCLBM_ENOMEM = -2,    /* caller arena too small, or allocation failed */
    MCLBM_EHIP = -3,      /* HIP runtime error */
    MCLBM_ESTATE = -4,    /* call out of order (e.g. step before init_fields) */
    MCLBM_EDIVERGED = -5  /* a monitor saw a non-finite density, velocity or C */
};
enum { MCLBM_D2Q9 = 0, MCLBM_D3Q19 = 1 };
enum { MCLBM_FORCING_GUO = 0, MCLBM_FORCING_SC = 1 };
/* Population storage.  *_SHIFT stores s_i = f_i - w_i * rhobar_s (rhobar_s =
 * fluid-mean density of component s at init_fields) in 16 bits with
 * round-to-nearest-even; collision arithmetic is FP32.  The solute is stored
 * unshifted.  F64 computes in FP64, the others in FP32. */
enum { MCLBM_F64 = 0, MCLBM_F32 = 1, MCLBM_F16_SHIFT = 2, MCLBM_BF16_SHIFT = 3 };
enum { MCLBM_SOLUTE_OFF = 0, MCLBM_SOLUTE_PERIODIC = 1, MCLBM_SOLUTE_INLET_OUTLET_X = 2 };

typedef struct {
    int32_t lattice;       /* MCLBM_D2Q9 or MCLBM_D3Q19 */
    int32_t nx, ny, nz;    /* >= 1; nz == 1 for D2Q9; ny, nz <= 65535 */
    int32_t ncomp;         /* 1 or 2 fluid components */
    int32_t forcing;       /* MCLBM_FORCING_* */
    int32_t solute;        /* MCLBM_SOLUTE_*; INLET_OUTLET_X needs nx >= 2 */
    int32_t storage;       /* MCLBM_F64 ... */
    int32_t monitor_every; /* K: monitors run after every step that is a multiple of K (>= 1) */
    int32_t reserved;      /* must be 0 */
    double tau[2];         /* BGK relaxation time per component, > 1/2 */
    double G[2][2];        /* cohesion matrix G_{s t} of eq:1.14 */
    double G_ads[2];       /* adhesion strength per component, eq:1.15 (< 0 wets) */
    double rho0;           /* pseudo-potential reference density, > 0 */
    double accel[3];       /* body force per unit density (force = rho_s * accel) */
    double D;              /* solute diffusivity, > 0 when the solute is on */
    double J0;             /* solute rest weight, in [0, 1) */
    double k_wall;         /* first-order wall reaction rate k = A exp(-E / R_u T), >= 0 */
    double C_in;           /* inlet concentration (INLET_OUTLET_X) */
    int32_t product;       /* 1: a second solute species (CO2) that every reacting wall link
                              produces at the reacting species' consumption rate k C_b
                              (eq:react, eq:reactCO2); needs the solute on; 0: off */
    int32_t rate_field;    /* 1: the reaction rate is a per-node field set with
                              mclbm_set_wall_rate (k_wall until then); 0: uniform k_wall */
    double D2;             /* product diffusivity, > 0 when the product is on */
    double C_in2;          /* product inlet concentration (INLET_OUTLET_X) */
    int32_t deposition;    /* 1: particle deposition (sec:particle_deposition, eq:surface_deposition):
                              the reacting solute species is the particle mass fraction C_p;
                              after every step each fluid node with a solid flow-lattice
                              neighbour adds dep_prob * C_p to its deposit C_ps, and the
                              nodes whose deposit exceeds 1 turn solid (see mclbm_step);
                              needs the solute on and a single lattice (not a batch); 0: off */
    int32_t reserved2;     /* must be 0 */
    double dep_prob;       /* deposition probability DP, > 0 when deposition is on */
} mclbm_params;

/* Device bytes the lattice needs for these parameters (populations A and B,
 * link words, pseudo-potentials, residual snapshot, staging, monitor
 * partials).  Returns MCLBM_EINVAL for invalid parameters. */
int mclbm_required_bytes(const mclbm_params* p, size_t* bytes);

/* Create a lattice for the problem of the multi-component LBM section: the
 * components with their own relaxation times (eq:1.16), the interaction
 * matrix G (eq:1.14), the adhesion strengths (eq:1.15), the pseudo-potential
 * reference density (eq:1.11), the forcing scheme (eq:1.17-eq:1.21) and the
 * solute of the reactive LBM (eq:therpop_species, eq:wetnode9).
 * device_arena: caller-owned device memory of at least
 * mclbm_required_bytes() bytes, 256-byte aligned, kept alive and untouched by
 * the caller until mclbm_destroy(); NULL makes the library allocate (and
 * later free) its own.  hip_stream: a hipStream_t (NULL = the null stream) on
 * which every kernel and copy of this handle is queued.  *out receives the
 * handle.  Errors: EINVAL (parameters: tau <= 1/2, bad dimensions or enums,
 * D <= 0 with the solute on, J0 outside [0, 1), k_wall < 0, rho0 <= 0,
 * monitor_every < 1, product or rate_field without the solute, D2 <= 0 with
 * the product, deposition without the solute or with dep_prob <= 0, nonzero
 * reserved fields), ENOMEM (arena too small), EHIP. */
int mclbm_init_lattice(const mclbm_params* p, void* device_arena, size_t arena_bytes,
                       void* hip_stream, mclbm_handle** out);

/* Set the solid geometry from a host mask of N bytes (1 = solid, 0 = fluid):
 * the solid indicator s(x) of the adhesion force (eq:1.15), the halfway
 * bounce-back links of the flow (eq:5 with the bounce-back rule of the
 * boundary-condition section) and the wet links of the solute (eq:wetnode9).
 * Fluid voxels that have solids on both sides along one axis (and, with the
 * inlet/outlet solute, voxels pinched against the x = 0 / x = nx-1 planes)
 * are reclassified as solid, to a fixed point; *n_reclassified (may be NULL)
 * receives their count.  Link words are rebuilt on the host and uploaded.
 * Invalidates the populations (call mclbm_init_fields next).
 * Errors: EINVAL if the mask is NULL or no fluid node remains. */
int mclbm_set_geometry(mclbm_handle* h, const uint8_t* solid_mask, int64_t* n_reclassified);

/* Copy out the geometry as the library uses it (each pointer may be NULL):
 * mask_out [N] bytes after reclassification; flow_links [N]: bit i set iff
 * fluid node n has a solid upstream node n - c_i (periodic); solute_links
 * [N]: bit k set iff solute link k of fluid node n is a wet (reactive) link,
 * i.e. n - e_k is solid and not across the x-planes in inlet/outlet mode.
 * Solid nodes report 0 links. */
int mclbm_get_geometry(mclbm_handle* h, uint8_t* mask_out, uint32_t* flow_links,
                       uint32_t* solute_links);

/* Initial state at equilibrium without force term: f_i = f^eq_i(rho_s, u)
 * of eq:6, h_k = h^eq_k(C, u) of eq:therpopeq_species.  rho: host FP64 [ncomp][N] (must be > 0 on fluid
 * nodes); u: host FP64 [3][N] or NULL (rest); C: host FP64 [N] or NULL
 * (zero).  The product species (if on) starts at zero concentration.
 * Resets the step counter and the residual snapshot, and fixes the
 * storage shift rhobar_s.  Errors: ESTATE before set_geometry, EINVAL. */
int mclbm_init_fields(mclbm_handle* h, const double* rho, const double* u, const double* C);

/* Per-node first-order reaction rate, e.g. k(x) = A exp(-E / (R_u T(x))) of a
 * prescribed temperature field (eq:reactO2): k_box is host FP64 [N] (box
 * nodes, x fastest; concatenated per sample for a batch), >= 0 and finite on
 * fluid nodes.  A reacting link uses the rate of its wall (wet) node.  Needs
 * rate_field = 1 and set_geometry first (set_geometry resets the field to
 * k_wall).  Errors: ESTATE (no rate field, or before set_geometry), EINVAL. */
int mclbm_set_wall_rate(mclbm_handle* h, const double* k_box);

/* Advance n >= 0 time steps (queued on the stream).  Monitors run after
 * every step whose index is a multiple of monitor_every; if any ran, the
 * call synchronises and returns MCLBM_EDIVERGED when the last one counted a
 * non-finite value.  Errors: ESTATE before init_fields, EINVAL (n < 0).
 *
 * With deposition on, every step is followed by the deposit update
 * (eq:surface_deposition).  If some deposit exceeds 1 after a step, those
 * nodes turn solid before the next step: the geometry is rebuilt as by
 * mclbm_set_geometry from the current solid mask plus those nodes (the pinch
 * rule applies again, and the nodes it fills turn solid too), the populations
 * and deposits of the remaining fluid nodes are carried over bit for bit, and
 * those of the new solid nodes are dropped.  Steps run in batches of up to 64
 * (never past a monitor step) with one synchronisation per batch; a batch in
 * which a conversion happened before its last step is rolled back to its
 * start and re-run up to that step (the result is the same as stepping one at
 * a time).  A per-node rate field set with mclbm_set_wall_rate is kept.  The
 * residual snapshot starts over after a conversion.  Graph replay is not used
 * with deposition.  Returns EINVAL (handle unusable) if deposition leaves no
 * fluid node. */
int mclbm_step(mclbm_handle* h, int64_t n);

/* Deposit C_ps of every box node (host FP64 [N], x fastest; 0 on solid nodes
 * and on nodes that never had a solid neighbour) and the number of nodes that
 * deposition has turned solid since init_fields (the pinch rule's included;
 * may be NULL).  Needs deposition = 1.  Errors: ESTATE before init_fields,
 * EINVAL. */
int mclbm_get_deposit(mclbm_handle* h, double* Cps, int64_t* converted);

/* Restore the deposits (host FP64 [N], box nodes; values at solid nodes are
 * ignored) and the converted-node count, e.g. from mclbm_get_deposit.  With
 * mclbm_get_geometry's mask, mclbm_get_populations(raw = 1) and these, a
 * deposition run resumes bit for bit: set_geometry(mask), init_fields,
 * set_populations(raw = 1), set_wall_rate if used, set_deposit.  With 16-bit
 * storage the raw values are relative to the storage shift that init_fields
 * fixes (the mean initial density over the fluid nodes), so init_fields must
 * give the same shift as in the original run (e.g. uniform initial densities).
 * Needs deposition = 1.  Errors: ESTATE before init_fields, EINVAL (negative or
 * non-finite deposit on a fluid node). */
int mclbm_set_deposit(mclbm_handle* h, const double* Cps, int64_t converted);

/* Macroscopic fields of the current (post-streaming) state: rho_s = sum_i f,
 * u = barycentric velocity with half force (eq:1.19, evaluated after
 * streaming), C = sum_k h_k.  rho: [ncomp][N], u: [3][N], C: [N], or [2][N]
 * (reacting species, then the product) when the product is on; any may be
 * NULL.  dst_is_device != 0: the pointers are device memory (no host sync
 * beyond the stream).  Solid nodes are 0. */
int mclbm_get_moments(mclbm_handle* h, double* rho, double* u, double* C, int32_t dst_is_device);

/* Latest monitor values (FP64, deterministic fixed-order reductions):
 * out[0] step of the monitor, out[1] mass of component 0, out[2] mass of
 * component 1 (0 if ncomp == 1), out[3] solute mass, out[4] r_u, out[5]
 * r_phi, out[6] r_C, out[7] non-finite count, out[8] fluid node count,
 * out[9] max(r_u, r_phi, r_C), out[10] current step; out[11..15] = 0.
 * Residual r_a = ||a(t) - a(t-K)||_2 / ||a(t)||_2 over fluid nodes, with
 * phi = (rho_0 - rho_1)/(rho_0 + rho_1); +inf before two monitors exist.
 * Fields absent from the run (phi with one component, C without solute)
 * report residual 0.  Before the first monitor out[0] = -1. */
int mclbm_get_monitors(mclbm_handle* h, double out[16]);

/* Run monitors now on the current state (as if at a monitor step). */
int mclbm_monitor_now(mclbm_handle* h);

/* Populations of the current pre-collision state (after streaming, before
 * the next collision).  raw == 0: FP64 decoded values [ncomp*Q + HS][N]
 * (flow [s][i], then solute [species][k]; HS = QS per solute species, 0
 * without solute, 2 QS with the product); raw != 0: the stored
 * bytes in the same order (8, 4 or 2 bytes per value; shifted values for
 * *_SHIFT).  Solid nodes read 0. */
int mclbm_get_populations(mclbm_handle* h, void* dst, int32_t raw);

/* Replace the pre-collision state of every sample (same layout as
 * mclbm_get_populations; the storage shift rhobar_s is kept).  Writing back
 * what get_populations(raw=1) returned continues the run bit for bit.
 * raw == 0: each FP64 value is encoded on the device by the store the step
 * kernels use: rounded to the arithmetic type (FP32 for F32 and the 16-bit
 * formats), the shift w_i rhobar_s of its flow plane subtracted in that type
 * (solute planes unshifted), then rounded to nearest even into FP16 / BF16
 * (Inf stays Inf, NaN stays NaN, overflow gives Inf).
 * Convergence flags of a batch and the residual snapshot start over.  ESTATE
 * before init_fields. */
int mclbm_set_populations(mclbm_handle* h, const void* src, int32_t raw);

/* Bytes of mclbm_get_populations output for the given raw flag. */
int mclbm_population_bytes(mclbm_handle* h, int32_t raw, size_t* bytes);

/* Step in chunks of monitor_every until the maximum residual at a monitor is
 * <= tol or max_steps have been taken.  *steps_taken (may be NULL) receives
 * the steps of this call.  In a batch each sample stops (is frozen, its state
 * kept) at the first monitor where its own residual is <= tol; a sample whose
 * monitor sees a non-finite value is frozen as diverged while the others go
 * on.  Returns MCLBM_OK when every sample converged, 1 when max_steps was
 * reached first, MCLBM_EDIVERGED when every sample has stopped and at least
 * one diverged (per-sample flags: mclbm_get_sample_monitors), or an error. */
int mclbm_run_to_residual(mclbm_handle* h, double tol, int64_t max_steps, int64_t* steps_taken);

/* Launch shape of the step kernels: block_threads per workgroup (64, 128 or
 * 256; default 256) and grid_blocks (0 = one pass over the fluid-node chunks,
 * default; else a persistent grid of that many workgroups, a multiple of 8,
 * that loops over the work list).  Every fluid node is updated by one thread
 * with the same arithmetic, so results do not depend on the launch shape. */
int mclbm_set_launch(mclbm_handle* h, int32_t block_threads, int32_t grid_blocks);

/* Addressing of the collide pass.  flat = 0 (default): raw buffer
 * instructions with 32-bit byte offsets whenever every population array, the
 * pseudo-potentials and each sample's node map are below 4 GiB, flat 64-bit addresses
 * otherwise; flat = 1: flat 64-bit addresses always.  Both forms store the
 * same values to the same elements (results are bit-identical); the buffer
 * form issues fewer instructions.  Drops captured graphs.  EINVAL for other
 * values. */
int mclbm_set_addressing(mclbm_handle* h, int32_t flat);

/* Number of y-bands of the fluid numbering (the fluid nodes of a sample are
 * numbered band by band, each band plane by plane, row by row, x fastest;
 * a band has at least 4 rows).  bands = 0 (default): eight, one per XCD;
 * else 1 .. 64.  With the geometry already set the fluid nodes are numbered
 * again at once, as by mclbm_set_geometry on the current masks: the fields
 * must be initialised again (ESTATE until init_fields), a per-node rate field
 * returns to k_wall and deposits to 0.  Results do not depend on the
 * numbering (every node takes the same arithmetic; only the order of the
 * monitors' reductions changes).  EINVAL outside 0 .. 64. */
int mclbm_set_bands(mclbm_handle* h, int32_t bands);

/* Time the step kernels over a set of numberings and launch shapes and keep
 * the fastest.  Launch shapes: block_threads 64, 128, 256 crossed with
 * grid_blocks 0 (one pass) and persistent grids of 8, 16 and 32 wavefronts
 * per compute unit.  Numberings: the current band count, and eight, four and
 * sixteen bands unless a per-node rate field, deposition or conjugate heat
 * transfer is on (numbering again would discard their state).  Each
 * candidate runs 2 untimed steps, then trial_steps (>= 1) steps timed with
 * HIP events on the handle's stream.  Needs set_geometry; it overwrites the
 * populations (uniform rest state, density 1), so init_fields must be called
 * afterwards (ESTATE until then).  The chosen numbering and shape are applied
 * as by mclbm_set_bands and mclbm_set_launch and returned in *bands,
 * *block_threads, *grid_blocks and *ms_per_step (any may be NULL).  The
 * candidates' timings are written to table[4 * i + 0..3] = (bands, block,
 * grid, ms per step) for i < table_rows (table may be NULL); *n_rows (may be
 * NULL) receives the number of candidates. */
int mclbm_autotune(mclbm_handle* h, int32_t trial_steps, int32_t* bands, int32_t* block_threads,
                   int32_t* grid_blocks, double* ms_per_step, double* table, int32_t table_rows, int32_t* n_rows);

/* enable != 0: run each aligned interval of monitor_every steps (which must
 * be even) as one replay of a captured HIP graph (the step kernels plus the
 * monitor), on a library-owned stream ordered after the caller's stream.
 * The graph is captured on first use, once a residual snapshot exists, and
 * dropped by set_geometry, init_fields, set_launch or set_graph. */
int mclbm_set_graph(mclbm_handle* h, int32_t enable);

/* ---------------------------------------------------------------------------
 * Batches of independent samples (for callers that run many small porous
 * samples at once).  The n samples share every parameter except nx, ny, nz
 * (EINVAL otherwise).  A batch handle accepts every call above; host arrays
 * are the per-sample arrays concatenated in sample order (sample s occupies
 * a block of fields * N_s values starting at fields * sum_{t<s} N_t), and
 * set_geometry takes the concatenated masks.  mclbm_run_to_residual stops
 * (freezes) each sample at the first monitor where its own maximum residual is
 * <= tol, keeps running the others, and returns MCLBM_OK when every sample has
 * converged.  mclbm_get_monitors then reports masses and counts summed over
 * samples and residuals maximised over the samples still running.  A single
 * lattice is a batch of one.  Deposition needs a batch of one (EINVAL). */
int mclbm_required_bytes_batch(const mclbm_params* p, int32_t n, size_t* bytes);
int mclbm_init_batch(const mclbm_params* p, int32_t n, void* device_arena, size_t arena_bytes,
                     void* hip_stream, mclbm_handle** out);

/* Monitors of sample s (layout of mclbm_get_monitors), plus out[11] = step
 * at which the sample converged in run_to_residual (-1 if not), out[12] = 1
 * if it is frozen and out[13] = step of the monitor at which it was found
 * diverged (-1 if not). */
int mclbm_get_sample_monitors(mclbm_handle* h, int32_t s, double out[16]);

/* Current step counter. */
int mclbm_get_step(mclbm_handle* h, int64_t* step);

/* Block until all queued work of the handle has finished. */
int mclbm_synchronize(mclbm_handle* h);

/* Free library-owned objects (never the caller's arena).  NULL is a no-op. */
/* ---------------------------------------------------------------------------
 * Conjugate heat transfer (Reactive LBM subsection).  Internal-energy
 * distributions on the flow lattice in the fluid (eq:therpop with the
 * equilibrium eq:therpopeq, advected by the barycentric velocity with half
 * force) and in the solid (eq:therpop_solid, eq:therpopeq_solid), coupled at
 * interface nodes -- fluid nodes with a solid flow-lattice neighbour, which
 * carry both distributions -- by the thermal counter-slip conditions
 * (eq:countSlipFluxCon, eq:countSlipTempCon: equal temperatures, heat-flux
 * balance with the reaction heat h_r k(T) C_b of eq:reacRate).  The unknown
 * populations of an interface node -- fluid ones whose upstream node is
 * solid; solid ones whose upstream node is a fluid node that is not an
 * interface node, or a fluid node while the downstream node is solid (the
 * solid field does not pass through the fluid) -- are w_i X_f and w_i X_s;
 * the two conditions give X_f and X_s (for a flat wall exactly
 * eq:unknownpopTempS and eq:unknownpopTempF).  The wet-link
 * reaction of the solute (eq:wetnode9, and the product's, eq:reactCO2) at an
 * interface node uses k(T) = A exp(-E_over_R / T) of the interface
 * temperature, and C_b and T are iterated per node until
 * |T_new - T| <= tol |T_new| (tol = max(T_tol, 4 x the arithmetic type's
 * epsilon)) or T_maxit iterations, before the step ends (the C_b - T loop of
 * the paper's flowchart).  Where the flux condition cannot be posed (every
 * missing fluid link of the node has a solid on both sides, possible only
 * along diagonals) the temperature condition alone is used and the solid
 * unknowns take the node's solid equilibrium; such nodes release no reaction
 * heat and are counted.  The thermal field is periodic in every direction. */
typedef struct {
    double tau_ef;    /* fluid energy relaxation time, 3 alpha_f + 1/2, > 1/2 */
    double tau_es;    /* solid energy relaxation time, 3 alpha_s + 1/2, > 1/2 */
    double rhocp_f;   /* rho c_p of the fluid, > 0 */
    double rhocp_s;   /* rho c_p of the solid, > 0 */
    double h_r;       /* heat released per unit of reacting species consumed, >= 0 */
    double A;         /* pre-exponential factor of k(T), >= 0 */
    double E_over_R;  /* activation temperature E / R_u of k(T), >= 0 */
    double T_tol;     /* relative tolerance of the interface iteration, > 0 */
    int32_t T_maxit;  /* iteration cap, >= 1 */
    int32_t reserved; /* must be 0 */
} mclbm_thermal;

/* Turn conjugate heat transfer on for a single lattice (not a batch) with F64
 * or F32 storage, without deposition or rate_field.  Call after init_lattice
 * and before set_geometry (the thermal node lists are built there; a call
 * after set_geometry resets the geometry: ESTATE until set_geometry again).
 * The thermal arrays are device memory the library allocates in
 * set_geometry and frees in destroy.  EINVAL for invalid values or an
 * unsupported combination. */
int mclbm_set_thermal(mclbm_handle* h, const mclbm_thermal* t);

/* Initial energy populations from a temperature field T [N] (host FP64, box
 * layout): fluid nodes the equilibrium eq:therpopeq at E = rho_c_p,f T and
 * velocity u ([3][N] host FP64, or NULL for rest), solid and interface nodes
 * w_i rho_c_p,s T; the interface iteration starts from T.  Call after
 * init_fields (which invalidates the thermal state: ESTATE from mclbm_step
 * until this call).  Resets the statistics of mclbm_get_thermal_stats. */
int mclbm_init_temperature(mclbm_handle* h, const double* T, const double* u);

/* Temperature [N] (host FP64): fluid and interface nodes E_f / rho_c_p,f,
 * solid nodes E_s / rho_c_p,s (E = sum of the node's energy populations). */
int mclbm_get_temperature(mclbm_handle* h, double* T);

/* Energy populations of the current state, FP64 host [Q][N] each, box layout:
 * g at fluid nodes (0 elsewhere), gs at solid and interface nodes (0
 * elsewhere).  Either pointer may be NULL. */
int mclbm_get_thermal_populations(mclbm_handle* h, double* g, double* gs);

/* Statistics since init_temperature: out[0] interface iterations in total,
 * out[1] interface solves that stopped at T_maxit without meeting the
 * tolerance, out[2] interface nodes where the flux condition cannot be posed
 * (a property of the geometry, counted once). */
int mclbm_get_thermal_stats(mclbm_handle* h, int64_t out[3]);

/* Practical HBM bandwidth of this device, measured with streaming kernels
 * (not part of the method: the ceiling the step kernels are compared with).
 * kind 0: read `bytes` of `a` (non-temporal 16-byte loads; `b` >= 4 KiB of
 * device memory receives nothing in practice); 1: write `bytes` to `a`;
 * 2: copy `bytes` from `a` to `b` (counted as read + write).  Grid:
 * blocks_per_cu x the device's CU count, 256 threads.  Runs iters + 1
 * passes on `stream` (the first untimed), synchronises, and returns the best
 * pass in *best_gbps (1e9 bytes/s).  `bytes` >= 4096 and a multiple of 16;
 * buffers are device memory owned by the caller.  EINVAL for bad arguments,
 * EHIP for a runtime error. */
int mclbm_hbm_probe(int32_t kind, void* a, void* b, size_t bytes, int32_t blocks_per_cu, int32_t iters,
                    void* stream, double* best_gbps);

void mclbm_destroy(mclbm_handle* h);

/* Message of the last failed call on h ("" if none); h == NULL gives the
 * message of the last failed mclbm_init_lattice / mclbm_required_bytes. */
const char* mclbm_last_error(const mclbm_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* MCLBM_H */
