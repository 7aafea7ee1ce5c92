/*
 * cgevap.h -- C-ABI of libcgevap.so: the time step of the two-component colour-gradient
 * lattice Boltzmann model with the reaction-limited evaporation sink of
 * Nath, Aouane & Harting, arXiv:2412.14859, on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *   - Every function returns a cge_status (0 = CGE_OK, < 0 = error) and never aborts or
 *     throws.  After an error, cge_last_error(ctx) holds a message (valid until the next
 *     call on that context).  Parameter errors are detected on the host before any device
 *     work, so they are testable without a GPU.
 *   - Large buffers are caller-owned DEVICE pointers (e.g. torch tensors on the GPU).  A
 *     context also needs scratch: per-block FP64 partials and small result buffers, which the
 *     library allocates at context creation and frees at cge_destroy, and large per-node
 *     scratch (the phase field, the moment and post-collision records of the split step and
 *     the record form, the fused step's second mask, the observables' phase field, the height
 *     flux's column sums; cge_scratch_bytes() in all), which cge_create allocates in one
 *     block and cge_create_with_scratch takes from the caller.
 *   - All device work is enqueued on the HIP stream given at cge_create, in order.
 *     Entry points that return host data (cge_observables, cge_timing) synchronise that
 *     stream; all others are asynchronous.
 *   - Node index n = x + nx*(y + ny*z); scalar fields are [nz][ny][nx], vector fields
 *     [D][nz][ny][nx], exported populations [2][Q][nz][ny][nx] with component 0 = red
 *     (the evaporating fluid) and component 1 = blue.  All axes are periodic; walls and
 *     obstacles are solid nodes given by the flags array.
 *   - Lattice directions (D2Q9):  0; +x; -x; +y; -y; (1,1); (-1,-1); (1,-1); (-1,1).
 *     (D3Q19): 0; +x; -x; +y; -y; +z; -z; then the xy, xz and yz diagonals, each in the
 *     order (+,+), (-,-), (+,-), (-,+).
 */
#ifndef CGEVAP_H
#define CGEVAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CGE_OK = 0,
    CGE_EINVAL = -1,       /* invalid argument or parameter                       */
    CGE_ENOMEM = -2,       /* device allocation of library scratch failed          */
    CGE_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed           */
    CGE_ESTATE = -4,       /* call out of order (e.g. step before cge_bind)        */
    CGE_EUNSUPPORTED = -5, /* valid but not supported combination                  */
    CGE_ENUMERIC = -6,     /* non-finite values found in the state                 */
    CGE_ECHECKPOINT = -7,  /* a saved state failed its integrity check             */
    CGE_ESCRATCH = -8      /* the grid needs more than the static scratch holds    */
} cge_status;

typedef enum { CGE_D2Q9 = 9, CGE_D3Q19 = 19 } cge_lattice;

/* Population storage.  FP64: doubles, FP64 arithmetic.  FP32S: floats holding shifted
 * values (see cge_bind), FP64 arithmetic in registers (the step is bandwidth-bound, and
 * FP32 arithmetic on near-uniform, quasi-steady fields repeats the same rounding at every
 * node every step, which drifts the component masses).  FP16S: half-precision storage of
 * the same shifted values with FP32 arithmetic (FP64 with cge_params.fp16_arith64) and
 * stochastic rounding on store. */
typedef enum { CGE_FP64 = 0, CGE_FP32S = 1, CGE_FP16S = 2 } cge_precision;

/* Evaporation-site rule.  GRAD_GT: ||F_{n-1}(x)|| > gamma with the colour gradient of the
 * previous step (Sec. II.B, site criterion and the remark after the method summary).
 * PHASE_LT: |rho^N(x)| < gamma from the current pre-sink phase field (a local variant).
 * SOFT: the sink is weighted by 1 / (1 + exp(-(||F_{n-1}(x)|| - gamma) / kappa)), a smooth
 * stand-in for GRAD_GT that makes the step differentiable in gamma (two-pass step only);
 * nodes with weight > 1/2 count as sites in the observables. */
typedef enum { CGE_SITE_GRAD_GT = 0, CGE_SITE_PHASE_LT = 1, CGE_SITE_SOFT = 2 } cge_site_rule;

/* Step implementation.
 *   TWOPASS: any lattice, geometry and relaxation times; writes the post-sink phase field to
 *            library scratch and pulls the populations twice.
 *   FUSED:   single pass, D3Q19, hard site rules, any relaxation times, no solid nodes or
 *            solid nodes only as whole z-planes with fluid on one side (floors and lids;
 *            CGE_EUNSUPPORTED at cge_create for D2Q9 or the SOFT rule, at cge_bind for other
 *            solid nodes); recomputes the phase field of each tile's halo.  Where the 19
 *            slots of one component exceed 4 GiB (32-bit buffer offsets) TWOPASS runs.
 *   SPLIT:   unit relaxation times (tau[0] == tau[1] == 1, else CGE_EUNSUPPORTED at
 *            cge_create), any lattice and geometry; the first pass writes the post-sink
 *            moments, the second finishes the step from them without re-reading populations.
 *   RECORD:  SPLIT's two passes, but between the steps of one cge_step call each node keeps
 *            a record of 14 values from which its post-collision populations follow at unit
 *            relaxation (post-sink density and phase field, velocity, colour gradient and
 *            the per-class coefficients of the equilibrium, perturbation (Eq. perturb) and
 *            recolouring (Eq. recolor)) instead of its 2Q populations.  The first step of
 *            a call pulls populations and the last writes them, so between calls the state
 *            is populations as for every other form; a call of one step is SPLIT's step.
 *            Same support as SPLIT.  The record is stored like the populations: FP64, FP32,
 *            or half precision with stochastic rounding at FP16S (then rebuilt in FP32), so
 *            the state between steps keeps the storage precision.  Needs 14 N values of
 *            library scratch in that type (rows padded to 256 B), allocated at cge_create for
 *            RECORD, and for AUTO where AUTO selects it.
 *   AUTO:    at unit relaxation times RECORD for D3Q19 and SPLIT for D2Q9 (where the record
 *            pull has no LDS-staged form and is no faster); otherwise FUSED where supported
 *            at FP32 or FP16 storage (at FP64 it is about three times slower), else TWOPASS.
 * All give the same results up to rounding. */
typedef enum {
    CGE_KERNEL_AUTO = 0,
    CGE_KERNEL_TWOPASS = 1,
    CGE_KERNEL_FUSED = 2,
    CGE_KERNEL_SPLIT = 3,
    CGE_KERNEL_RECORD = 4
} cge_kernel;

typedef struct {
    int lattice;            /* cge_lattice                                               */
    int nx, ny, nz;         /* nodes per axis, >= 1 (ny, nz <= 65535); nz == 1 for D2Q9  */
    int precision;          /* cge_precision                                             */
    double rho_in[2];       /* bulk densities of red and blue; define alpha_k (Sec. II.A) */
    double tau[2];          /* relaxation times, > 1/2 (Sec. II.A)                        */
    double sigma;           /* surface tension in the perturbation operator (Eq. perturb) */
    double beta;            /* recolouring parameter in [0, 1] (Eq. recolor)              */
    double phi;             /* uniform mass flux when no flux field is bound (Sec. II.B)  */
    double sbar;            /* layer factor Sbar >= 1 (Eq. relation)                      */
    double gamma;           /* site threshold Gamma (site criterion)                      */
    double kappa;           /* width of the soft site rule, > 0 (CGE_SITE_SOFT only)      */
    int site_rule;          /* cge_site_rule                                              */
    int kernel;             /* cge_kernel                                                 */
    unsigned long long seed; /* stochastic-rounding stream (FP16S only)                   */
    double recolor_fade;    /* 0 (default): cos(theta_i) = F.c_i / (||F|| ||c_i||) as in     */
                            /* Eq. recolor, taken as 0 where F.F <= 1e-24 (with the         */
                            /* perturbation).  w > 0: an optional regularisation, not the   */
                            /* paper's model, multiplies cos(theta_i) by                    */
                            /* clamp(||F||/w - 1, 0, 1) (for small periodic boxes where F   */
                            /* vanishes by symmetry at mixed nodes).  Must be finite, >= 0. */
    int fp16_arith64;       /* CGE_FP16S only: 0 (default) FP32 arithmetic on the half       */
                            /* storage; 1 FP64 arithmetic.  FP32 arithmetic repeats its       */
                            /* rounding at every bulk node and step, which moves red mass at  */
                            /* the interface steadily into the blue (the 256^3 drop loses 51 %*/
                            /* more volume over 10000 steps at phi = 1e-5); FP64 arithmetic   */
                            /* removes that drift and costs about 11 % of the step.  Must be  */
                            /* 0 for the other precisions.                                    */
} cge_params;

/* Observables of the current state (post-streaming, pre-sink), reduced in FP64 in a fixed
 * order over fluid nodes. */
typedef struct {
    long long step;         /* steps taken since the last init / counter reset            */
    long long n_sites;      /* sites the next step will use                               */
    long long v_half;       /* #nodes with rho_r > max(rho_r)/2 (interface, Sec. III)     */
    long long n_negative;   /* #populations f_i^k < -1e-6 rho_k^in t_i(alpha_k) (negative */
                            /* beyond rounding noise; the sink can drive f_0^r below 0)   */
    long long site_steps;   /* cumulative number of (site, step) sink applications        */
    double mass_r, mass_b;  /* total red and blue mass                                    */
    double sink_total;      /* cumulative mass moved red -> blue by the sink              */
    double v_mass;          /* mass_r / rho_in[0]                                         */
    double perim_sites;     /* n_sites / sbar: interface measure seen by the sink         */
    double perim_grad;      /* (1/2) sum ||grad rho^N||: interface measure of rho^N       */
    double max_u;           /* max |u|                                                    */
    double p_in, p_out;     /* mean EOS pressure over rho^N > 0.9 and < -0.9 (Eq. EOS)    */
    double max_rho_r;       /* max rho_r                                                  */
} cge_obs;

typedef struct cge_ctx cge_ctx;

/* Validate parameters, allocate the library scratch on the current HIP device, and attach
 * the HIP stream (hipStream_t passed as void*, NULL = default stream).
 * Errors: CGE_EINVAL (bad parameters; *out untouched), CGE_EUNSUPPORTED (a step form that
 * does not support the parameters), CGE_ENOMEM, CGE_EDEVICE. */
cge_status cge_create(const cge_params* params, void* hip_stream, cge_ctx** out);

/* Bytes of the large per-node scratch a context of these parameters uses (0 for invalid
 * parameters): at D3Q19 256^3 about 8 (phase field) + 1 (mask) + 16 (moments) + 56 (records)
 * + 8 (observables) + 1 (column sums) bytes per node at FP32 storage. */
size_t cge_scratch_bytes(const cge_params* params);

/* cge_create with the large scratch in a caller-owned device buffer of at least
 * cge_scratch_bytes() bytes, 256-byte aligned, which must stay valid and unused by others
 * until cge_destroy (the library never frees it); the library then allocates only its
 * per-block partials and result buffers.  CGE_EINVAL for a NULL, smaller or misaligned
 * buffer; otherwise as cge_create. */
cge_status cge_create_with_scratch(const cge_params* params, void* hip_stream, void* scratch,
                                   size_t scratch_bytes, cge_ctx** out);

/* Bytes of one population buffer: 2*Q*nx*ny*nz elements of 8 (FP64), 4 (FP32S) or
 * 2 (FP16S) bytes.  Returns 0 for invalid parameters. */
size_t cge_population_bytes(const cge_params* params);

/* Attach caller-owned device buffers (they must stay valid while the context uses them).
 *   pop_a, pop_b : two population buffers of cge_population_bytes() each (ping-pong).
 *                  Their content is an internal encoding: per direction i the colour-blind
 *                  deviation f_i^r + f_i^b - rho_in[1] t_i(alpha_b) and the colour
 *                  difference f_i^r - f_i^b of the post-collision values, stored so that
 *                  streaming is a pull.  Use cge_set/get_populations to convert.
 *   carry        : the site data carried to the next step: nx*ny*nz bytes, 1 where the next
 *                  step evaporates (site mask; it may be overwritten between steps to impose
 *                  a site set), or for CGE_SITE_SOFT nx*ny*nz doubles holding ||F_{n-1}||.
 *   flags        : nullable, nx*ny*nz bytes, nonzero = solid node (halfway bounce-back,
 *                  neutral wetting).  Not changed by the library.
 *   phi_field    : nullable, nx*ny*nz per-node fluxes phi(x) (double for FP64, float for
 *                  FP32S/FP16S); replaces params.phi (sink s = phi(x)/sbar per step).
 * Errors: CGE_EINVAL for a NULL ctx/pop_a/pop_b/carry or pop_a == pop_b. */
cge_status cge_bind(cge_ctx* ctx, void* pop_a, void* pop_b, unsigned char* carry,
                    const unsigned char* flags, const void* phi_field);

/* Equilibrium initial state from device FP64 fields rho_r, rho_b ([N]) and u ([D][N],
 * nullable = rest):  f_i^k = rho_k [t_i(alpha_k) + W_i (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)]
 * (Eq. feq per component).  Also sets the site mask from the gradient of the initial
 * phase field and zeroes the step and sink counters.  Requires cge_bind. */
cge_status cge_init_equilibrium(cge_ctx* ctx, const double* rho_r, const double* rho_b,
                                const double* u);

/* Load / export the state as device FP64 populations [2][Q][N] (post-streaming, pre-sink,
 * plain f^r and f^b).  Solid nodes export zeros and are ignored on load.  Loading does not
 * touch the site mask or counters (see cge_reset_sites, cge_set_counters). */
cge_status cge_set_populations(cge_ctx* ctx, const double* f);
cge_status cge_get_populations(cge_ctx* ctx, double* f);

/* Snapshot of the state in the library's own encoding (bitwise exact round trip), for
 * checkpoint / resume; cge_state_bytes() bytes of device memory at dst / src (256-byte
 * aligned).  Layout:
 *   [0, pb)            the current population buffer, pb = cge_population_bytes()
 *   [coff, coff + cb)  the carried site data, coff = pb rounded up to 256, cb its size
 *   [toff, toff + 32)  an integrity trailer, toff = coff + cb rounded up to 256: four
 *                      little-endian uint64: magic 0x5441545356454743, a fingerprint of the
 *                      parameters, pb + cb, and a checksum
 * checksum = sum mod 2^64, over the 8-byte little-endian words w_i of the populations and then
 * of the site data (each region zero-padded to a multiple of 8 bytes; i counts on from the
 * first region into the second), of m(w_i XOR (i * 0xD6E8FEB86659FD93)), where m(z) is the
 * splitmix64 step: z += 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
 * z = (z ^ z>>27) * 0x94D049BB133111EB; m = z ^ z>>31.
 * fingerprint = 64-bit FNV-1a over the bytes of int32 lattice, nx, ny, nz, precision,
 * site_rule, then float64 rho_in[0], rho_in[1], then int32 1 (format version).
 * cge_save_state writes all of it (asynchronously).  cge_load_state first recomputes the
 * checksum of src on the device and compares the trailer (synchronising the stream), and
 * returns CGE_ECHECKPOINT, leaving the state untouched, for a missing trailer, a trailer of
 * other parameters or a checksum mismatch.  Counters are not included (see
 * cge_set_counters). */
size_t cge_state_bytes(const cge_params* params);
cge_status cge_save_state(cge_ctx* ctx, void* dst);
cge_status cge_load_state(cge_ctx* ctx, const void* src);

/* The same integrity check on a snapshot copied to HOST memory (cge_state_bytes() bytes), with
 * no device work: CGE_OK, CGE_ECHECKPOINT, or CGE_EINVAL for bad parameters or NULL. */
cge_status cge_verify_state(const cge_params* params, const void* snapshot);

/* Adjoint (reverse mode) of nsteps steps, for the site rules GRAD_GT (sites held at those of
 * the forward run) and SOFT, with or without solid nodes (the transposes of the halfway
 * bounce-back and of the neutral-wetting value are included).  The loss is given through its
 * derivatives with respect to the final phase field rho^N_T (e.g. 2 (rho^N_T - target) for a
 * squared mismatch) and the final density rho_T (e.g. rho_T/2 and (1 + rho^N_T)/2 together
 * for the red mass), and the gradients with respect to the flux field phi(x) and the site
 * threshold Gamma are returned.
 *   cge_forward_ckpt : from the current state, advance nsteps and save the state (as
 *                      cge_save_state) at steps 0, K, 2K, ... into ckpt[0..ceil(nsteps/K)-1]
 *                      and the state after nsteps into ckpt[ceil(nsteps/K)], each buffer of
 *                      cge_state_bytes().  At unit relaxation times it steps with the split
 *                      form (CGE_KERNEL_SPLIT), which the backward recomputes with.
 *   cge_backward     : call after cge_forward_ckpt with the same nsteps, K and checkpoints
 *                      (again as often as needed, e.g. for another loss).  seg:
 *                      cge_segment_bytes(K) bytes for the
 *                      recomputed steps of one segment (at unit relaxation times each step's
 *                      phase field, moments and site data, otherwise each state);
 *                      work: cge_adjoint_bytes();
 *                      dL_drhoN, dL_drho: [N] doubles, either may be NULL (read as zero) but
 *                      not both; their values at solid nodes are ignored (solid nodes hold no
 *                      state); grad_phi (out): [N] doubles, dL/dphi(x) summed
 *                      over the steps (phi held over time); grad_phi_t (out, nullable):
 *                      [nsteps][N] doubles, dL/dphi(x, t) per step; grad_gamma (host, nullable):
 *                      dL/dGamma (0 for GRAD_GT).  All buffers except grad_gamma are device
 *                      memory.  Forward states are recomputed from the checkpoints; on return
 *                      the context holds the state after nsteps again, with its step counter
 *                      and sink bookkeeping.
 * Errors: CGE_EINVAL (missing buffers, nsteps or K < 1), CGE_EUNSUPPORTED (PHASE_LT rule,
 * height flux or outlets on), CGE_ECHECKPOINT (a checkpoint fails the integrity check of
 * cge_load_state; the context then holds an intermediate state: load one), CGE_EDEVICE. */
size_t cge_adjoint_bytes(const cge_params* params);
size_t cge_segment_bytes(const cge_params* params, int K);
cge_status cge_forward_ckpt(cge_ctx* ctx, long long nsteps, int K, void* const* ckpt);
cge_status cge_backward(cge_ctx* ctx, long long nsteps, int K, void* const* ckpt, void* seg,
                        void* work, const double* dL_drhoN, const double* dL_drho,
                        double* grad_phi, double* grad_phi_t, double* grad_gamma);

/* Recompute the site mask from the current state (gradient of its phase field). */
cge_status cge_reset_sites(cge_ctx* ctx);

/* Change the site threshold Gamma (and, for the SOFT rule, the width kappa > 0; pass
 * kappa <= 0 to keep it) of a live context; later steps use the new values.  Under GRAD_GT the
 * carried mask was taken with the old Gamma: call cge_reset_sites or load a state to retake
 * it.  CGE_EINVAL for a non-finite value. */
cge_status cge_set_site_threshold(cge_ctx* ctx, double gamma, double kappa);

/* Height-dependent flux (Sec. III, space- and time-varying flux; Eq. heated): with every > 0
 * the bound flux field is overwritten, before every step whose step counter is a multiple of
 * `every`, with phi(x) = phi_s / (K + h / h_scale), where h is the drop height of x's column
 * along the last lattice axis (z for D3Q19, y for D2Q9; the substrate normal): the sum over the
 * column's fluid nodes of the red fraction (1 + rho^N)/2 of the current pre-sink state.  The
 * field depends on the current state only, so resumed runs take the same fluxes.  every <= 0
 * switches it off (the field keeps its last values).  Each refresh reads the whole state once.
 * The column sums (8 bytes per 8 nodes of a column) live in the context's scratch.
 * Needs a bound flux field (CGE_ESTATE otherwise); CGE_EINVAL unless K > 0, h_scale > 0 and
 * phi_s is finite.  The adjoint does not differentiate through the heights: cge_forward_ckpt
 * and cge_backward return CGE_EUNSUPPORTED while it is on. */
cge_status cge_set_height_flux(cge_ctx* ctx, double phi_s, double K, double h_scale,
                               long long every);

/* Pressure outlets for the blue component (Zou and He; Sec. III, density contrast) on the end
 * planes of the last lattice axis (z for D3Q19, y for D2Q9): lo switches the plane at index 0,
 * hi the plane at the last index.  At an outlet node the populations entering through the
 * plane are replaced by those that hold the blue density at rho_out with no tangential
 * velocity (normal velocity from the known populations); no red fluid enters (its entering
 * populations are 0).  The values are taken at once for the current state, after every step,
 * and after cge_init_equilibrium and cge_set_populations (cge_load_state restores a state as
 * saved).  Solid nodes on a plane are left alone.  lo = hi = 0 switches the outlets off.
 * CGE_EINVAL for rho_out <= 0 or not finite, or fewer than 3 planes along the axis.  The
 * adjoint returns CGE_EUNSUPPORTED while outlets are on. */
cge_status cge_set_outlet(cge_ctx* ctx, int lo, int hi, double rho_out);

/* Launch shape of the z-marching kernels (the record form's pull for D3Q19 at every precision,
 * the fused step): planes per z-chunk of a block's march.  0 (the default) chooses it from the grid
 * (and, for the record pull, the device's compute-unit count); planes > 0 takes that many
 * (at most nz).  Results do not depend on it beyond the grouping of the FP64 sink partials
 * (1e-15 relative).  For tuning, and for tests of chunked marches on small grids.
 * CGE_EINVAL for planes < 0. */
cge_status cge_set_zchunk(cge_ctx* ctx, int planes);

/* Restore the step counter and the FP64 sink bookkeeping (checkpoint resume). */
cge_status cge_set_counters(cge_ctx* ctx, long long step, long long site_steps,
                            double sink_total);

/* Advance nsteps >= 0 time steps (method summary of Sec. II.B: sink rate, sites, mass
 * exchange, moments, collision, perturbation, recolouring, streaming). */
cge_status cge_step(cge_ctx* ctx, long long nsteps);

/* Reduce the observables of the current state into *out (host).  Synchronises the stream. */
cge_status cge_observables(cge_ctx* ctx, cge_obs* out);

/* The observables of cge_observables for a state given by buffers instead of a context, for
 * callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation).  It allocates nothing: its scratch (per-block FP64
 * partials and an FP64 phase field) is a static 64 MiB device array of the library, which each
 * GPU it runs on holds until the process ends; a grid qualifies when
 *     8 (12 B + N) + 256 <= 64 MiB,   N = nx ny nz,  B = ceil(nx / min(256, 64 ceil(nx/64))) ny nz
 * (D3Q19 up to 199^3, D2Q9 up to about 2800^2), else CGE_ESCRATCH before any device work.
 *   params : the state's lattice, grid, precision and physics (validated as by cge_create)
 *   pop    : device, one population buffer in the library's encoding (cge_bind), e.g. the
 *            first cge_population_bytes() bytes of a cge_save_state snapshot
 *   carry  : device, the carried site data of that state (the snapshot's carry part)
 *   flags  : device, nullable, solid nodes as for cge_bind
 *   out    : device, one cge_obs written by the last kernel; step, site_steps and sink_total
 *            (context bookkeeping) are written as 0.  Copy it to the host after the stream.
 * All work is enqueued on hip_stream (NULL = default stream); nothing synchronises.  Every call
 * on one GPU shares that GPU's scratch, and a call overwrites all of it that it reads, so
 * consecutive calls need no clearing, but calls that overlap on one GPU (different streams or
 * host threads) race and must be serialised by the caller.  The first call on a device looks
 * up the scratch address there (hipGetSymbolAddress).  Errors: CGE_EINVAL (bad parameters or a
 * NULL pop, carry or out), CGE_ESCRATCH, CGE_EDEVICE. */
cge_status cge_observables_noalloc(const cge_params* params, const void* pop,
                                   const unsigned char* carry, const unsigned char* flags,
                                   void* hip_stream, cge_obs* out);

/* Per-node FP64 fields of the current state into device arrays (each nullable):
 * rho_r, rho_b, rhoN ([N]) and u ([D][N]).  Solid nodes get 0 (rhoN: wetting value). */
cge_status cge_fields(cge_ctx* ctx, double* rho_r, double* rho_b, double* u, double* rhoN);

/* Kernel timing: when on, HIP events on the context's stream mark the start of every step
 * and the end of each of its passes.  cge_timing synchronises and returns the summed
 * milliseconds and the number of timed steps since timing was switched on; cge_timing_kernel
 * the milliseconds and launches of one pass kernel by name (e.g. "k_pull_record_zm",
 * "k_finish_record", "k_moments", "k_finish", "k_finish_tile", "k_pull_record", "k_phase",
 * "k_collide", "k_fused"; a pass's helper launches, such as the wetting of solid nodes,
 * count with it), 0 and 0 for a kernel that has not run. */
cge_status cge_set_timing(cge_ctx* ctx, int on);
cge_status cge_timing(cge_ctx* ctx, double* total_ms, long long* steps);
cge_status cge_timing_kernel(cge_ctx* ctx, const char* kernel, double* total_ms,
                             long long* launches);

/* Name of the step kernel the context launches (static string). */
const char* cge_kernel_name(const cge_ctx* ctx);

/* Lattice tables of the library (host): W, A, B, C (Q doubles each, t_i(a) = A_i + B_i a,
 * C_i the perturbation constants), c (3Q ints), opp (Q ints), zeta.  Any pointer may be NULL. */
cge_status cge_lattice_tables(int lattice, double* W, double* A, double* B, double* C, int* c,
                              int* opp, double* zeta);

/* Plain device-to-device copy of nbytes with a streaming kernel on hip_stream (bandwidth
 * reference for the roofline).  Pointers must be 16-byte aligned. */
cge_status cge_copy_probe(void* dst, const void* src, size_t nbytes, void* hip_stream);

const char* cge_last_error(const cge_ctx* ctx);
void cge_destroy(cge_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CGEVAP_H */
