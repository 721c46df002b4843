/*
 * demag.h -- C ABI of the MI355X (gfx950) demagnetizing-field engine.
 *
 * The library evaluates the demagnetizing field of Eq. (1) (Sec. II),
 *     H_d,i = - sum_j N(i - j) . M_j      (sum over every mesh cell, j = i included),
 * on a single GPU as a zero-padded 3-D FFT convolution (Sec. II, Fig. 1, App. A),
 * and advances the LLG equation (Eq. 5, Sec. III) and the atomistic stochastic
 * LLG equation at T = 0 (Eq. 10, Sec. IV) with it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Field arrays (M, H, m, S) are caller-owned DEVICE pointers to contiguous
 *    FP32 data laid out structure-of-arrays as [3][nz][ny][nx] (component, z, y,
 *    x; x fastest).  Nothing is copied; the library never frees them.
 *  - Units are SI: M and H in A/m, lengths in m, gamma in m/(A s), J in J.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call except
 *    the *_setup / *_destroy calls only enqueues work on that stream and returns;
 *    the caller synchronises.  Plans own their device workspace, so one plan must
 *    not be used by two streams at the same time.
 *  - Every call returns a status code (DEMAG_OK = 0 or a negative DEMAG_E*).
 *    No exception, exit or abort crosses the ABI.  demag_last_error() returns a
 *    thread-local, human-readable message describing the last failure on the
 *    calling thread.  A failed call leaves its outputs unspecified but the plan
 *    usable unless the status is DEMAG_EHIP (a HIP runtime failure).
 *  - Mesh sizes: every n_d must be 1 or a power of two, n_x and n_y at most 2048
 *    and n_z at most 128 (larger or other sizes return DEMAG_EUNSUPPORTED).
 *    n_x and n_y may also be F 2^j with F = 3, 5 or 15 and j >= 1 (6, 10, 30,
 *    ..., 480, 960, 1920): the transforms then add radix-3 and radix-5 passes;
 *    such meshes take DEMAG_FP32 with open boundaries (other flags return
 *    DEMAG_EUNSUPPORTED).  The padded transform length is N_d = 2 n_d, or 1
 *    when n_d = 1 (n_d along a periodic axis).
 */
#ifndef DEMAG_H
#define DEMAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    DEMAG_OK = 0,
    DEMAG_EINVAL = -1,        /* bad argument (null pointer, size <= 0, non-finite cell) */
    DEMAG_ENOMEM = -2,        /* device allocation failed or budget exceeded */
    DEMAG_EUNSUPPORTED = -3,  /* mesh size the kernels do not implement */
    DEMAG_EHIP = -4,          /* a HIP runtime call failed */
    DEMAG_EBUSY = -5          /* serving: request not finished / queue full */
};

/* ---- plan flags --------------------------------------------------------- */
enum {
    DEMAG_FP32 = 0,           /* FP32 FFT stages (default) */
    /* The radix-16 passes of every FFT stage as BF16 matrix products on the
     * matrix cores: each 16-point DFT of a batch of 32 is one real 32x32 DFT
     * matrix times the 32 x 32 block of input real/imaginary parts, both
     * split into BF16 terms (v = v0 + v1 [+ v2]) and the leading cross
     * products accumulated in FP32; twiddles, passes of radix < 16, the
     * tensor product and all data stay FP32.  Same result definition and
     * tolerance as DEMAG_FP32. */
    /* Two-term split (3 products per DFT step): REFUSED by demag_setup with
     * DEMAG_EUNSUPPORTED (demag_plan_bytes returns 0).  Its error follows the
     * largest spectral values, so where the field is small against them (a
     * few sparse sources seen from far away) it exceeds rel-L2 2e-5 (6.4e-4
     * measured on a 1024x1024x32 film with 400 sources).  The value stays
     * reserved so that it is never reused for another meaning. */
    DEMAG_BF16X2_MFMA = 1,
    DEMAG_BF16X3_MFMA = 2,    /* three-term split, 6 products per DFT step */
    /* May be or-ed with the others: demag_field accepts H == M (the field
     * overwrites the magnetisation).  Every form reads all of M into the plan's
     * spectral workspace in its first kernel and writes H in its last, in
     * stream order, so the aliasing is safe; without the flag H == M is
     * refused as a likely mistake. */
    DEMAG_INPLACE = 4,
    /* May be or-ed with one of the above.  llg_step evaluates H_d once per RK4
     * step, at the step start, and takes the values at the sub-steps
     * (t + dt/2 twice, t + dt) from the quartic in time through the five most
     * recent step-start fields: the polynomial extrapolation of the
     * demagnetizing field of Sec. III (quartic for RK4).  The first five steps
     * of a trajectory, and every step after a change of dt, evaluate all four
     * stages.  The history (5 x 12 N bytes) lives in the plan and is allocated
     * on the first llg_step; llg_reset discards it. */
    DEMAG_EXTRAPOLATE_HD = 8,
    /* May be or-ed with the others.  The kernel is the point-dipole tensor of
     * Eq. (8), N_ab(r) = V (delta_ab |r|^2 - 3 r_a r_b) / (4 pi |r|^5) with
     * N(0) = 0 and V = dx dy dz, instead of the cell-averaged tensor: with
     * M = mu_B mu_S S^ / V per lattice site, demag_field returns the lattice
     * dipole-dipole field of Eq. (8) (an atom plan with macro = 1 and this
     * flag steps the full dipole-dipole interaction). */
    DEMAG_POINT_DIPOLE = 16,
    /* Periodic boundary conditions (Sec. II: a modified kernel and no zero
     * padding along a periodic axis).  May be or-ed with DEMAG_FP32 (only) and
     * the flags above; atom plans and the server take open meshes only.  Along
     * a periodic axis d the transform has length n_d (circular convolution)
     * and the tensor is the sum over the body's periodic images,
     *   N_pbc(r) = sum_m N(r + m_x n_x dx e_x + m_y n_y dy e_y + m_z n_z dz e_z),
     * |m_d| <= P on periodic axes (0 on open ones), P = DEMAG_PBC_IMAGES value
     * (0: the mesh alone, folded), taken at the displacements
     * r_d in (-n_d/2, n_d/2]; a component odd in d (N_xy odd in x and y, ...)
     * is set to 0 at r_d = n_d/2, the value the infinite image sum has there.
     * Images farther than 64 max(dx, dy, dz) use the moment expansion of the
     * cell-pair tensor through its h^2 term (relative error below 1e-6 there).
     * llg_step wraps the exchange stencil around periodic axes.  Set-up cost
     * grows as (2P + 1)^(periodic axes) FP64 tensor evaluations per octant
     * entry. */
    DEMAG_PBC_X = 32,
    DEMAG_PBC_Y = 64,
    DEMAG_PBC_Z = 128
};
/* Image count P (0..255) of a periodic plan, in bits 8..15 of the flags. */
#define DEMAG_PBC_IMAGES_SHIFT 8
#define DEMAG_PBC_IMAGES(p) (((uint32_t)(p) & 0xffu) << DEMAG_PBC_IMAGES_SHIFT)

/* Mesh of n_x x n_y x n_z rectangular cells of size dx x dy x dz (m). */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
} demag_mesh;

typedef struct demag_plan demag_plan;   /* opaque; owns N^ and the FFT workspace */

/*
 * demag_setup -- build a plan for one mesh: computes the transformed
 * demagnetizing tensor N^ (the "convolution kernel" of App. A, computed at
 * initialisation as in Sec. II) in FP64 on the GPU, stores its six independent
 * real components in FP32 packed by the y and z symmetries, and allocates the
 * FFT workspace.
 *   mesh    in   mesh description (copied).
 *   flags   in   DEMAG_FP32 or DEMAG_BF16X3_MFMA (DEMAG_BF16X2_MFMA is refused),
 *                optionally or-ed with DEMAG_INPLACE, DEMAG_EXTRAPOLATE_HD and
 *                DEMAG_POINT_DIPOLE;
 *                with DEMAG_FP32 also DEMAG_PBC_X/Y/Z | DEMAG_PBC_IMAGES(P).
 *   stream  in   hipStream_t used for the set-up kernels; the call synchronises it.
 *   out     out  receives the new plan (NULL on failure).
 * Errors: EINVAL (null/invalid mesh), EUNSUPPORTED (size), ENOMEM, EHIP.
 */
int demag_setup(const demag_mesh* mesh, uint32_t flags, void* stream, demag_plan** out);

/*
 * demag_field -- H = H_d(M) of Eq. (1): x R2C -> y FFT -> (z FFT, N^.M^, z IFFT)
 * -> y IFFT -> x C2R (App. A execution order, without the inter-GPU transfers).
 *   M  in   device, FP32 [3][nz][ny][nx], A/m.
 *   H  out  device, FP32 [3][nz][ny][nx], A/m; may be M only for a plan set up
 *           with DEMAG_INPLACE.
 * Errors: EINVAL (null plan/pointer, H == M without DEMAG_INPLACE), EHIP.
 */
int demag_field(demag_plan* plan, const float* M, float* H, void* stream);

/* Bytes of device memory a plan for `mesh` holds (N^ + FFT workspace), for
 * budget-based admission. Returns 0 for an invalid or unsupported mesh. */
size_t demag_plan_bytes(const demag_mesh* mesh, uint32_t flags);

/*
 * demag_get_kernel -- copy the packed FP32 transformed tensor into `dst`
 * (device), laid out [6][Z1][X1][Y1] with components (xx, yy, zz, xy, xz, yz)
 * and D1 = N_d/2 + 1 (1 when N_d = 1).  The stored value already includes the
 * factor -1/(N_x N_y N_z) of Eq. (1) and the unnormalised inverse transforms.
 * `count` is the capacity of dst in floats; returns EINVAL if too small.
 */
int demag_get_kernel(demag_plan* plan, float* dst, size_t count, void* stream);

int demag_destroy(demag_plan* plan);

/* ---- micromagnetic LLG (Eqs. 4, 5; RK4 of Sec. III) --------------------- */
/* The integrator is chosen by the entry point, not by a parameter field:
 * llg_step always integrates with classic RK4 (the micromagnetic scheme of
 * Sec. III) and atom_step always with Heun (the atomistic scheme of Sec. IV),
 * so neither parameter struct carries an integrator selector. */
typedef struct {
    double Ms;        /* saturation magnetisation, A/m (> 0) */
    double A;         /* exchange stiffness, J/m (Eq. 4) */
    double alpha;     /* Gilbert damping (>= 0) */
    double gamma;     /* gyromagnetic ratio, m/(A s) (> 0) */
    double Hzee[3];   /* constant applied field, A/m */
} llg_params;

/*
 * llg_step -- advance the unit magnetisation m by `nsteps` classic RK4 steps of
 * the LLG equation in Landau-Lifshitz form,
 *     dm/dt = -gamma/(1+alpha^2) [m x H_eff + alpha m x (m x H_eff)],
 * with H_eff = H_d(Ms m) + 2A/(mu0 Ms) lap(m) + Hzee (free boundaries; Eq. 4),
 * H_d recomputed at every RK stage, and |m| renormalised at the end of each step.
 *   m       in/out device FP32 [3][nz][ny][nx], unit vectors, updated in place.
 * With nsteps >= 2 (no DEMAG_EXTRAPOLATE_HD, timing off) one step is captured
 * as a HIP graph on a plan-private stream and replayed nsteps times on
 * `stream`; the capture is kept in the plan and redone when m, the parameters,
 * dt, the chunk count or a tile variant change.  The launches are those of
 * single steps, so the result is bitwise the same; small meshes, whose steps
 * are bound by launch overhead, gain most.
 * Errors: EINVAL (null, nsteps < 0, dt not finite, bad params), ENOMEM, EHIP.
 */
int llg_step(demag_plan* plan, float* m, const llg_params* params, double dt,
             int32_t nsteps, void* stream);

/*
 * llg_step_noalloc -- the steps of llg_step for callers that cannot allocate
 * device memory: code under HIP stream capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arithmetic and launches as llg_step
 * stepping one by one, so m comes out bitwise the same; the steps are launched
 * eagerly (no graph), and the plan must already exist (demag_setup allocates).
 * The RK4 stage buffers (12 N floats) are a fixed 64 MiB device array in the
 * library, one copy per GPU held until the process ends, so
 *   N <= llg_noalloc_max_cells() = 1,398,101 cells.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams or threads) race and must be serialised by the caller.
 *   m       in/out device FP32 [3][nz][ny][nx], unit vectors, updated in place.
 * Errors: EINVAL (null, nsteps < 0, dt not finite, bad params, mesh above the
 * limit, current device not the plan's), EUNSUPPORTED (DEMAG_EXTRAPOLATE_HD
 * plans, which keep an H_d history), EHIP.
 */
int llg_step_noalloc(demag_plan* plan, float* m, const llg_params* params, double dt,
                     int32_t nsteps, void* stream);
/* The largest mesh (cells) llg_step_noalloc accepts. */
size_t llg_noalloc_max_cells(void);

/*
 * llg_reset -- discard the H_d history of a DEMAG_EXTRAPOLATE_HD plan, so that
 * the next llg_step starts a new trajectory (call it after setting m to a state
 * that does not continue the previous steps).  No effect on other plans.
 * Errors: EINVAL (NULL plan).
 */
int llg_reset(demag_plan* plan);

/*
 * demag_field_mean -- out[c] = mean over the plan's cells of component c of the
 * field v (c = x, y, z): the average magnetization <m> recorded along a
 * trajectory in the precision study of Sec. II (Fig. 2).  FP64 partial sums in
 * a fixed order, so the value is reproducible bit for bit.
 *   v    in   device, FP32 [3][nz][ny][nx].
 *   out  out  device, 3 FP32 values; written on `stream` (no synchronisation).
 * Errors: EINVAL (null argument), EHIP.
 */
int demag_field_mean(demag_plan* plan, const float* v, float* out, void* stream);

/* ---- atomistic spin dynamics (Eqs. 7, 9, 10; Sec. IV) ------------------- */
typedef struct {
    int32_t nx, ny, nz;   /* spins on a simple-cubic lattice */
    double a;             /* lattice constant, m */
    int32_t macro;        /* macrocell edge in spins (N_S = macro^3); must divide n_d */
} atom_mesh;

typedef struct {
    double J;             /* nearest-neighbour exchange energy, J (Eq. 7) */
    double mu_s;          /* spin moment in Bohr magnetons */
    double alpha, gamma;
    double Hzee[3];
} atom_params;

typedef struct atom_plan atom_plan;   /* owns a demag_plan on the macrocell mesh */

/* atom_setup -- plan for a lattice; the demagnetizing field is evaluated on the
 * spin-averaged macrocell mesh (Eq. 9) of edge h = macro * a. */
int atom_setup(const atom_mesh* mesh, uint32_t flags, void* stream, atom_plan** out);

/*
 * atom_step -- `nsteps` Heun steps of Eq. (10) at T = 0 for the unit spins S:
 * H = J/(mu0 mu_B mu_s) sum_nn S_j (Eq. 7, open boundaries)
 *   + H_d of the spin's macrocell (Eq. 9 then Eq. 1) + Hzee;
 * predictor S + dt f(S), corrector S + dt/2 (f(S) + f(S_p)), renormalised at
 * the end of each step.
 *   S  in/out device FP32 [3][nz][ny][nx] unit vectors, updated in place.
 */
int atom_step(atom_plan* plan, float* S, const atom_params* params, double dt,
              int32_t nsteps, void* stream);

int atom_destroy(atom_plan* plan);

/* ---- per-stage timing (tracing) ----------------------------------------- */
/* Kernel stages a plan launches, in pipeline order. */
enum {
    DEMAG_STAGE_X_FWD = 0,    /* x R2C (+ transposed store) */
    DEMAG_STAGE_Y_FWD = 1,    /* y FFT */
    DEMAG_STAGE_Z_CONV = 2,   /* z FFT, N^.M^, z IFFT */
    DEMAG_STAGE_Y_INV = 3,    /* y IFFT */
    DEMAG_STAGE_X_INV = 4,    /* x C2R */
    DEMAG_STAGE_LLG = 5,      /* exchange + LLG RK4 stage update */
    DEMAG_NSTAGES = 6
};

/*
 * demag_timing_enable -- when max_records > 0, every later stage launch of this
 * plan is bracketed by a pair of HIP events on its stream (up to max_records
 * launches per stage; further launches are not timed).  0 disables timing and
 * frees the events.  Each timed launch takes a record's two events
 * (hipExtLaunchKernelGGL), so they hold the kernel's own start and end, as a
 * kernel trace sees them.  They still lengthen the gaps between kernels a
 * little (about 0.07 ms per RK4 step of 16 kernels on 512 x 512 x 16 cells),
 * so time whole steps or evaluations with timing disabled.  llg_step with
 * nsteps >= 2 replays its captured step only while timing is disabled.
 */
int demag_timing_enable(demag_plan* plan, int32_t max_records);

/*
 * demag_timing_read -- waits for the recorded events, writes the summed elapsed
 * time (ms) and the number of timed launches of each stage into
 * total_ms[DEMAG_NSTAGES] and launches[DEMAG_NSTAGES], and clears the records.
 */
int demag_timing_read(demag_plan* plan, double* total_ms, int32_t* launches);

/* ---- tile-shape variants and autotuning ---------------------------------- */
/*
 * Each FFT stage (DEMAG_STAGE_X_FWD .. DEMAG_STAGE_X_INV) has DEMAG_NVARIANTS
 * tile shapes (how many rows, lines or columns one workgroup transforms).  All
 * variants of the five-pass stages produce bit-identical results; they differ
 * only in speed.  (At N_z = 64 the five-pass Z_CONV variants 0 and 2 are a
 * register form of the z convolution with 32 or 64 columns per workgroup and
 * variant 1 the LDS form; they run the same per-column arithmetic.  For long x
 * rows, X_FWD variant 0 takes variant 2's rows on twice the threads.)  In the
 * thin-mesh form (DEMAG_FORM_THIN) the variant of
 * X_FWD and X_INV sets the row pairs one workgroup transforms per round (8, 4
 * or 2; 4, 2 or 1 at n_x = 1024), again bit-identical, and the variant of
 * Z_CONV, where n_y >= 256, the y convolution's thread count (radix order) and
 * columns per workgroup: variant 0 takes 128 threads (1024 = 16 8 8; n_y <= 512),
 * 1 takes 256 threads (1024 = 16 16 4) and one column, 2 takes 256 threads and
 * the two mirror planes kz, N_z - kz of a column, with the second column's
 * loads in flight while the first is transformed.  Variants 1 and 2 give the
 * same bits; variant 0 rounds differently.  Each is deterministic and within
 * the 2e-5 contract.
 * demag_autotune times every variant of every stage inside whole evaluations on
 * the plan's own buffers (HIP events around the stage's launches, two rounds of
 * 3 evaluations; synchronises `stream`; earlier per-stage timing records of the
 * plan are dropped, its timing capacity kept), keeps the fastest and
 * remembers the choice for later plans of the same mesh size in this process
 * (the serving engine's plans included).  Plans made with a BF16 MFMA flag
 * always run the middle tile shape (variant 1, whatever is set);
 * demag_autotune then tunes only the chunk count.
 */
enum { DEMAG_NVARIANTS = 3 };
int demag_autotune(demag_plan* plan, void* stream);

/*
 * The y FFT, z convolution and y IFFT run chunk by chunk over the n_x + 1 kx
 * planes of the spectrum through a re-used buffer of at most 128 MB (so a
 * chunk's spectra stay in the 256 MB Infinity Cache).  demag_autotune also picks
 * the number of chunks; demag_set_chunks sets it explicitly (at least
 * ceil((n_x + 1) / planes the buffer holds), at most n_x + 1).  The result does
 * not depend on the chunking.
 */
int demag_set_chunks(demag_plan* plan, int32_t nchunks);
int demag_get_chunks(demag_plan* plan, int32_t* nchunks);
int demag_set_variant(demag_plan* plan, int32_t stage, int32_t variant);
int demag_get_variant(demag_plan* plan, int32_t stage, int32_t* variant);

/*
 * demag_get_form -- which kernel sequence the plan runs (fixed at set-up):
 *   DEMAG_FORM_FIVE_PASS   x R2C, y FFT, z convolution, y IFFT, x C2R
 *                          (stages X_FWD, Y_FWD, Z_CONV, Y_INV, X_INV);
 *   DEMAG_FORM_THIN        FP32 plans of thin meshes (32 <= n_x <= 1024,
 *                          16 <= n_y <= 1024, n_z <= 16, powers of two, open
 *                          boundaries): x R2C with the z FFT (timed as X_FWD),
 *                          y FFT + tensor product + y IFFT (timed as Z_CONV),
 *                          z IFFT with the x C2R (X_INV).  The chunk count has
 *                          no effect.
 * Both compute the same H (Eq. 1) to FP32 rounding.
 *   plan  in   plan;   form  out  one of the values below.
 * Errors: EINVAL (NULL argument).
 */
enum { DEMAG_FORM_FIVE_PASS = 5, DEMAG_FORM_THIN = 3 };
int demag_get_form(demag_plan* plan, int32_t* form);

/* ---- serving: continuous batching of independent LLG simulations --------- */
/*
 * A server owns a worker thread and a HIP stream.  Requests (a mesh, LLG
 * parameters, dt, a number of RK4 steps and an initial magnetisation in host
 * memory) are queued by serve_submit and admitted while the device memory they
 * need (FFT workspace, RK4 buffers, m, and the transformed tensor of their mesh
 * unless an active request already holds it) fits the HBM budget and fewer than
 * max_active requests run.  Every iteration advances all active requests by the
 * same number of RK4 steps with shared launches (requests of equal transform
 * lengths share each FFT-stage launch; one launch updates every mesh's LLG
 * stage); finished requests are copied back to host memory, their memory is
 * released and queued requests are admitted.  Each result is bit-identical to
 * running the same request alone with llg_step.
 */
typedef struct demag_server demag_server;

enum {
    SERVE_GRAPHS = 1          /* replay each active set's step from a captured HIP graph */
};

typedef struct {
    uint64_t submitted, completed, failed;
    int32_t active, queued;
    double cell_steps;        /* sum over completed requests of cells x steps */
    size_t bytes_in_use, peak_bytes;
    uint64_t iterations;      /* worker iterations that advanced active requests */
    uint64_t graph_captures;  /* graphs captured (one per distinct active set) */
} serve_stats;

/* hbm_budget_bytes: device memory the server may hold for requests (> 0);
 * max_active: requests advanced together (1 .. 1024); flags: SERVE_GRAPHS or 0. */
int serve_open(size_t hbm_budget_bytes, int32_t max_active, uint32_t flags, demag_server** out);

/* Queues a request; copies mesh, params and m0 (host, FP32 [3][nz][ny][nx], unit
 * vectors) and returns immediately with its id.  Errors: EINVAL, EUNSUPPORTED. */
int serve_submit(demag_server* srv, const demag_mesh* mesh, const llg_params* params, double dt,
                 int32_t nsteps, const float* m0_host, uint64_t* request_id);

/* Blocks until the request finishes; copies m (host, same layout as m0) and the
 * latency from submission to completion (seconds, may be NULL), then forgets
 * the request.  Returns the request's status (ENOMEM if it can never fit the
 * budget, or the error that stopped it). */
int serve_wait(demag_server* srv, uint64_t request_id, float* m_out_host, double* latency_s);

int serve_get_stats(demag_server* srv, serve_stats* out);

/* Stops the worker after the current iteration; unfinished requests are dropped. */
int serve_close(demag_server* srv);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* demag_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DEMAG_H */
