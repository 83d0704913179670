/*
 * ddm.h -- C-ABI of libddm, an MI355X (gfx950) implementation of the additive
 * overlapping domain decomposition method (DDM) for the Helmholtz equation of
 * W. Leng and L. Ju, "An Additive Overlapping Domain Decomposition Method for
 * the Helmholtz Equation" (arXiv 1807.04180).
 *
 * Problem (Sec. 1 eq. helm, Sec. 3.1 eq. PMLweak0): the truncated PML problem
 *     J^{-1} div(A grad u) + k(x)^2 u = f   on the box extended by the PML,
 *     u = 0 on its boundary,
 * with A = diag(alpha_2/alpha_1, alpha_1/alpha_2) (3D analogue), J = prod
 * alpha_j, alpha_j = 1 + i sigma_j (Sec. 2.1), discretised by the 5-point
 * (2D) / 7-point (3D) finite-difference scheme on a uniform mesh (Sec. 4).
 *
 * Grid: per axis the physical interval [0, M h] has M cells; the unknowns
 * are the nodes g = -n_pml+1 .. M+n_pml-1 (M + 2 n_pml - 1 of them) with
 * Dirichlet nodes at g = -n_pml and g = M + n_pml, and sigma(x) =
 * sigma0 (t/n_pml)^2, t = distance in cells outside [0, M].  Global vectors
 * are row-major [nrhs][z][y][x] over the unknowns ("nglob" entries per RHS).
 *
 * Partition (Sec. 2.2, Sec. 3.1): N[d] subdomains per axis, cores of
 * C = M/N cells (half-open; the first and last also hold the global PML);
 * every interior side of a subdomain is extended by n_ov overlap cells with
 * sigma = 0 and n_pml PML cells (the shifted profile of eq. PMLprofile).
 * "Packed" vectors hold one vector per subdomain box: [nrhs][subdomain a]
 * [box, x fastest]; ddm_geometry gives each box and its offset.
 *
 * Every pointer argument named f, u, g, uhat, U, r, out is a DEVICE pointer
 * (HIP global memory, e.g. from a torch tensor), complex128 interleaved;
 * relres / norms / info are HOST pointers.  The caller owns all of them;
 * the library owns its factors and workspaces (freed by ddm_destroy).  All
 * work is enqueued on the stream given to ddm_setup; calls that return host
 * values synchronise that stream before returning.
 *
 * Errors: every call returns 0 on success, a negative code on a hard error
 * (nothing useful was written) and a positive code on a soft one (outputs
 * hold the best result reached).  ddm_last_error gives a message.  No C++
 * exception crosses this boundary.
 */
#ifndef DDM_H
#define DDM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DDM_OK = 0,
    DDM_EINVAL = -1,      /* bad argument, layout or non-finite input         */
    DDM_ENOMEM = -2,      /* device allocation failed or HBM budget exceeded  */
    DDM_ESINGULAR = -3,   /* zero / tiny pivot in a subdomain block          */
    DDM_EHIP = -4,        /* HIP runtime error                                */
    DDM_ESTATE = -5,      /* call out of order (e.g. iterate before factor)  */
    DDM_ENOCONV = 1,      /* tolerance not reached within maxiter            */
    DDM_EDIVERGED = 2     /* residual grew by more than 1e6 over its minimum */
};

typedef enum { DDM_FP64 = 0, DDM_MIXED = 1 } ddm_precision;
typedef enum { DDM_STATIONARY = 0, DDM_FGMRES = 1 } ddm_method;

typedef struct {
    int dim;                  /* 2 or 3                                          */
    int M[3];                 /* interior cells per axis (unused axes ignored)   */
    double h;                 /* mesh size (equal on all axes)                   */
    int n_pml;                /* PML cells, >= 2                                  */
    double sigma0;            /* PML strength (alpha = 1 + i sigma), >= 0; must
                                 be 0 when reflection > 0                       */
    int N[3];                 /* subdomains per axis; M[d] % N[d] == 0            */
    int n_ov;                 /* overlap cells (the d~ of Sec. 2.2), >= 2;
                                 core width M/N >= n_ov + 2 when N > 1          */
    ddm_precision precision;  /* DDM_FP64: everything in complex128.
                                 DDM_MIXED: subdomain factors, local solves and
                                 transfers in complex64; residual, assembly and
                                 the outer Krylov / refinement in FP64.          */
    size_t hbm_budget_bytes;  /* 0 = no limit; else ddm_setup refuses a plan
                                 larger than this (DDM_ENOMEM)                   */
    double reflection;        /* 0: use sigma0 as given.  In (0, 1): the PML
                                 strength is derived from this target reflection
                                 of the quadratic profile (the sigma~ of Sec.
                                 2.1 is left open by the paper; this is the
                                 round-trip reading): a wave of the smallest
                                 wave number k_ref = sqrt(min k^2) crossing the
                                 layer twice is damped by exp(-2 k_ref sigma0
                                 n_pml h / 3) = reflection, i.e.
                                 sigma0 = 3 ln(1/reflection) / (2 k_ref n_pml h).
                                 ddm_pml_strength returns the value used.       */
    int k2_on_host;           /* ddm_setup's k2 is a HOST pointer when != 0, a
                                 DEVICE pointer when 0                           */
} ddm_problem;

typedef struct {
    ddm_method method;   /* DDM_STATIONARY: Algorithm 3.1 continued as an
                            iterative solver (Sec. 4.2.1); DDM_FGMRES: flexible
                            GMRES right-preconditioned by K DDM steps
                            (Sec. 4.2.2)                                       */
    double tol;          /* stop when ||f - L u||_2 / ||f||_2 <= tol (per RHS) */
    int maxiter;         /* max DDM steps (stationary) / Arnoldi steps (FGMRES)*/
    int restart;         /* FGMRES restart length (e.g. 30)                    */
    int K;               /* DDM steps per preconditioner application; 0 means
                            N1 + N2 (+ N3)                                     */
    int refine_every;    /* DDM_MIXED stationary: restart the c64 DDM on the
                            FP64 residual after this many steps without a 2x
                            gain (0 = never; the residual-corrected sources
                            make restarts unnecessary in practice)             */
    int check_every;     /* DDM_STATIONARY: test the stopping criterion (and
                            synchronise with the host) after every
                            check_every-th step only (0 or 1 = every step).
                            A right-hand side that meets tol stops at the
                            first checked step at or after that point; the
                            iteration count reported is that step.  Between
                            checks the steps are only enqueued: the host
                            neither waits for nor reads the residual norms.
                            The last step (maxiter) is always checked.        */
} ddm_solve_opts;

typedef struct {
    int iters;           /* DDM steps (stationary) or Arnoldi steps (FGMRES)  */
    int local_solves;    /* local solves per subdomain (n_Local_Solve)         */
    double relres;       /* final FP64 relative residual                      */
    double seconds;      /* wall time of the solve                            */
    int status;          /* DDM_OK / DDM_ENOCONV / DDM_EDIVERGED for this RHS */
} ddm_rhs_info;

typedef struct ddm_handle ddm_handle;

/* Peak device bytes of a handle for at most nrhs_max right-hand sides per
 * call, for admission control: everything ddm_setup allocates (tables,
 * factors, step workspaces, the handle-owned copies of f and u used by the
 * step graphs and the slots) plus the factorisation workspace that
 * ddm_factor holds while it runs.  DDM_FGMRES solves allocate their Krylov
 * basis (2 restart + 1 global vectors per RHS) on first use, on top of this,
 * and refuse it with DDM_ENOMEM when it would exceed hbm_budget_bytes.
 * Returns DDM_EINVAL for an invalid problem. */
int ddm_memory_required(const ddm_problem *p, int nrhs_max, size_t *bytes);

/* Build the discretisation and partition tables (Sec. 3.1, Sec. 2.2) and
 * allocate device memory for up to nrhs_max right-hand sides per call.
 * k2: k(x)^2 on the global unknown grid (double, nglob entries, row-major
 * [z][y][x]), a DEVICE pointer, or a HOST pointer when p->k2_on_host != 0;
 * copied, so the caller may free it afterwards.  DDM_EINVAL for non-finite
 * entries, and for reflection > 0 with sigma0 != 0, reflection >= 1 or a
 * non-positive minimum of k2.  stream: hipStream_t (NULL = default stream).
 * On success *out receives a handle. */
int ddm_setup(const ddm_problem *p, const double *k2, int nrhs_max, void *stream, ddm_handle **out);

/* PML strength sigma0 the handle uses (given, or derived from reflection). */
int ddm_pml_strength(const ddm_handle *h, double *sigma0);

/* Factor every subdomain operator L_{i,j} of Algorithm 3.1 once (the direct
 * local solver of Sec. 4) as a block-tridiagonal LU with grid-line (2D) /
 * grid-plane (3D) blocks: S_l = D_l - C_l S_{l-1}^{-1} B_{l-1}, stored as
 * W_l = S_l^{-1} (complex128 for DDM_FP64, complex64 for DDM_MIXED).
 * Returns DDM_ESINGULAR if a block pivot vanishes. */
int ddm_factor(ddm_handle *h);

/* Run nsteps steps of Algorithm 3.1 from a zero state for nrhs sources f
 * (nrhs x nglob) and write the DDM iterate u = sum_a beta_{0;a} U_a
 * (eq. tsum) after the last step.  relres (host, nsteps x nrhs, may be NULL)
 * receives ||f - L u|| / ||f|| after every step. */
int ddm_iterate(ddm_handle *h, const void *f, void *u, int nrhs, int nsteps, double *relres);

/* Solve L u = f to opts->tol with the DDM as iterative solver or as FGMRES
 * preconditioner (Sec. 4.2).  info (host, nrhs entries, may be NULL) gets the
 * per-RHS outcome.  Returns DDM_OK when every RHS converged, else the worst
 * per-RHS status. */
int ddm_solve(ddm_handle *h, const void *f, void *u, int nrhs, const ddm_solve_opts *opts,
              ddm_rhs_info *info);

/* Text of the last error on this handle (or of the last failed ddm_setup
 * when h is NULL).  Valid until the next call on the handle. */
const char *ddm_last_error(const ddm_handle *h);

/* Release all device memory of the handle. */
void ddm_destroy(ddm_handle *h);

/* ---- geometry and single-row entry points (Sec. 2.2 / Alg. 3.1 steps) ---- */

/* Device memory of the handle (host pointers, may be NULL): *held = bytes it
 * holds now, *peak = the most it held at once since ddm_setup (the
 * factorisation workspace included). */
int ddm_device_bytes(const ddm_handle *h, size_t *held, size_t *peak);

/* Sizes: out[0] = nglob, out[1] = packed size per RHS (sum of |E_a|),
 * out[2] = number of subdomains, out[3] = factor bytes. */
int ddm_sizes(const ddm_handle *h, long *out);

/* Boxes of subdomain a in physical node indices: out[0..2] core low,
 * out[3..5] core high, out[6..8] extended-box low, out[9..11] extended-box
 * high (unused axes 0), out[12] packed offset, out[13] box size. */
int ddm_geometry(const ddm_handle *h, int a, long *out);

/* out = L_h u on the global grid (the 5/7-point PML operator). */
int ddm_apply(ddm_handle *h, const void *u, void *out, int nrhs);

/* r = f - L_h u (r may be NULL) and per-RHS squared 2-norms of r and f,
 * summed in FP64 in a fixed order (host arrays, nrhs entries each). */
int ddm_residual(ddm_handle *h, const void *f, const void *u, void *r, int nrhs,
                 double *rnorm2, double *fnorm2);

/* ddm_residual for callers that cannot allocate device memory or synchronise
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * allocation): the same kernels and results (bit for bit), but it allocates
 * nothing, creates no events and does not wait.  norms is a DEVICE array of
 * 2 nrhs doubles: norms[q] = ||r_q||^2, norms[nrhs + q] = ||f_q||^2, written
 * on the handle's stream.  The block partial sums live in one static device
 * array of the library (1 MiB, 2 nrhs x (grid rows rounded up to 8) doubles
 * at most; larger calls return DDM_EINVAL and say the limit), held by every
 * GPU the library has run on until the process ends and shared by all calls
 * on that GPU: calls that overlap on one GPU race.  Never profiled. */
int ddm_residual_noalloc(ddm_handle *h, const void *f, const void *u, void *r, int nrhs,
                         double *norms);

/* Step-1 sources: g_a = f restricted to the core of a (f_{i,j} of Sec. 2.2),
 * written to the packed vector g (zero outside the cores). */
int ddm_restrict_core(ddm_handle *h, const void *f, void *g, int nrhs);

/* Local solves of one step: uhat_a = L_a^{-1} g_a for every subdomain a and
 * RHS (packed in, packed out; may alias).  Requires ddm_factor.  With
 * DDM_MIXED the solve runs in complex64 and is widened on output. */
int ddm_local_solve(ddm_handle *h, const void *g, void *uhat, int nrhs);

/* Source transfer of Sec. 2.2 / eq. talg_2: g_a = sum over the 8 (2D) / 26
 * (3D) neighbours b of Psi_{b->a}(uhat_b), Psi_{b->a}(v) = -L_a(beta_{b->a}
 * v) restricted to chi_{b->a}; edge / face neighbours read lag1, corner /
 * edge neighbours lag2, 3D vertex neighbours lag3 (packed; NULL = zero). */
int ddm_transfer(ddm_handle *h, const void *lag1, const void *lag2, const void *lag3, void *g,
                 int nrhs);

/* Assembly of eq. tsum: u = sum_a beta_{0;a} U_a (packed U in, global u out). */
int ddm_assemble(ddm_handle *h, const void *U, void *u, int nrhs);

/* ---- continuous batching (slots) -------------------------------------------- */
/* The handle's nrhs_max right-hand-side positions are slots that requests can
 * join and leave at step boundaries while the others keep iterating: each
 * slot runs Algorithm 3.1 from its own first step (its source, its own step
 * count) on the shared factors.  Slot arithmetic does not depend on the other
 * slots, so a slot's result is the same alone and in any mix. */

/* Start a solve in a free slot: f is one DEVICE global vector (nglob
 * complex128).  The slot's iterate starts at zero; its first step uses f
 * restricted to the cores.  Returns DDM_EINVAL if the slot is in use. */
int ddm_slot_admit(ddm_handle *h, int slot, const void *f);

/* Enqueue nsteps DDM steps for every occupied slot (asynchronous). */
int ddm_slots_step(ddm_handle *h, int nsteps);

/* Synchronise and report per slot (nrhs_max entries each, host): relres of
 * the slot's current iterate (-1 for a free slot) and its step count. */
int ddm_slots_poll(ddm_handle *h, double *relres, int *steps);

/* Copy a slot's iterate to u (DEVICE, nglob complex128; may be NULL) and free
 * the slot.  ddm_iterate / ddm_solve return DDM_ESTATE while any slot of the
 * handle is occupied (they share its buffers). */
int ddm_slot_retire(ddm_handle *h, int slot, void *u);

/* ---- observability -------------------------------------------------------- */

/* Kernel classes of one DDM step. */
enum { DDM_K_SUBST = 0, DDM_K_TRANSFER = 1, DDM_K_ASSEMBLE = 2, DDM_K_RESIDUAL = 3, DDM_K_NCLASS = 4 };

typedef struct {
    long launches[DDM_K_NCLASS];  /* kernel launches recorded                   */
    double ms[DDM_K_NCLASS];      /* summed GPU time between the HIP events that
                                     bracket each launch on the handle's stream */
    double bytes[DDM_K_NCLASS];   /* algorithmic HBM bytes of those launches:
                                     substitution = every stored block inverse
                                     read once per sweep plus the block vectors
                                     it reads and writes                        */
} ddm_profile;

/* Start (on != 0, counters reset) or stop recording per-launch HIP events. */
int ddm_profile_enable(ddm_handle *h, int on);

/* Synchronise the stream and return the counters since the last enable. */
int ddm_profile_read(ddm_handle *h, ddm_profile *out);

/* ---- tuning --------------------------------------------------------------- */

/* Block-substitution kernel variants (the local solves of every DDM step):
 *   0  one launch per block index over all subdomains (any block size; only
 *      with the one-directional factor layout);
 *   1  one workgroup per elimination chain walking all its blocks, the block
 *      recurrence kept on chip (block size <= 256).  With the twisted layout
 *      (default when 2 nsub workgroups fit on the device's compute units, at
 *      most 128 subdomains on a 256-CU MI355X) every subdomain has two
 *      chains that meet once at a middle block;
 *   2  two workgroups per chain of the twisted layout, each taking half of
 *      every block's columns and exchanging partial sums with its partner
 *      once per block (block size <= 256, all 4 nsub workgroups resident:
 *      at most 64 subdomains on a 256-CU MI355X, RHS in tiles of up to 4):
 *      for problems with fewer chains than CUs;
 *   3  one workgroup per chain as in 1, one wave per 16-row tile of every
 *      block, the products W_l V on the matrix cores (MFMA 16x16x4, f32 for
 *      DDM_MIXED, f64 for DDM_FP64) for tiles of 16 right-hand sides (fewer
 *      are padded with zeros): each inverse is read once per sweep and 16
 *      RHS.  The inverses are stored in this kernel's operand order, so
 *      selecting it (or leaving it) re-runs the factorisation of a factored
 *      handle.  Block size <= 256; default when nrhs_max >= 8. */
enum { DDM_SOLVE_PERLINE = 0, DDM_SOLVE_CHAIN = 1, DDM_SOLVE_CHAIN2 = 2, DDM_SOLVE_MMA = 3, DDM_SOLVE_NVARIANTS = 4 };

/* Factor layout: twisted != 0 eliminates every subdomain from both ends
 * towards a middle block (two chains per subdomain), 0 from the first block
 * on.  Default: twisted when every chain can have its own compute unit
 * (2 nsub <= CUs: at most 128 subdomains on MI355X).  Changing it
 * discards the factors (call ddm_factor again). */
int ddm_set_factor_layout(ddm_handle *h, int twisted);

/* Select a variant; DDM_EINVAL if it does not apply to this problem.  A
 * switch to or from DDM_SOLVE_MMA re-factorises a factored handle (its
 * status is returned: DDM_ESINGULAR etc.). */
int ddm_set_solve_variant(ddm_handle *h, int variant);

/* Currently selected variant. */
int ddm_get_solve_variant(const ddm_handle *h);

/* Time every applicable variant on nrhs right-hand sides (reps local solves
 * each, after one warm-up) and keep the fastest (re-factorising when the
 * layout of the inverses changes, see DDM_SOLVE_MMA).  times_ms (host, may be
 * NULL, DDM_SOLVE_NVARIANTS entries) receives the mean time per local solve,
 * -1 for variants that do not apply or could not be launched. */
int ddm_autotune(ddm_handle *h, int nrhs, int reps, double *times_ms);

/* RHS tile of the chain variant (DDM_SOLVE_CHAIN) for calls of more than 4
 * right-hand sides: 4 (1024-thread workgroups), 8 (512 threads for
 * DDM_FP64, 1024 for DDM_MIXED) or 16 (the default choice for 16 or more
 * RHS); 0 restores the choice by batch size.  The tile can change the
 * rounding of a result (a different order of partial sums).  Exposed for
 * the autotuner; DDM_EINVAL for other values. */
int ddm_set_chain_tile(ddm_handle *h, int rt);

/* Mean time of one local solve (all subdomains, nrhs right-hand sides of
 * zeros in the handle's workspace) with the current variant, layout and
 * tile: one warm-up, then reps solves timed with HIP events on the handle's
 * stream (host ms, synchronises).  For the autotuner. */
int ddm_time_local_solve(ddm_handle *h, int nrhs, int reps, double *ms);

/* Replay the steady-state step of the stationary solve (transfer, local
 * solves, accumulation, residual and norms) as a captured hipGraph, one per
 * generation of the ring of local solutions (default on).  The handle then
 * iterates on its own copies of f and u.  Capture falls back to plain
 * launches where it is unavailable. */
int ddm_set_graphs(ddm_handle *h, int on);

/* Number of step-graph launches since setup (observability). */
long ddm_graph_launches(const ddm_handle *h);

/* Bound on the spin iterations of the wait of one chain for its partner at
 * the middle block (default 2^22).  When a wait exceeds it the launch drains
 * without waiting and the call reports DDM_EHIP.  Exposed so that this
 * failure path can be exercised from the host. */
int ddm_set_spin_limit(ddm_handle *h, int limit);

/* Form of the transferred sources Psi_{b->a}(v) (every transfer: ddm_transfer,
 * the stationary step, the FGMRES preconditioner, the slots).
 *   DDM_TRANSFER_DIRECT (default): -L_a(beta_{b->a} v) on chi_{b->a}
 *       (the transfer operators of Sec. 2.2);
 *   DDM_TRANSFER_PHI: -(L_a(beta v) - beta L_a v) on chi_{b->a}, the
 *       discrete counterpart of the Phi form of eq. Phi (the remark after the
 *       horizontal transfer in Sec. 2.2): first differences of beta times v,
 *       without the wave number.  It equals the direct form wherever L_a v
 *       vanishes on the support of beta.  The DDM's local solutions satisfy
 *       that only when the subdomains lie along one axis (N > 1 on one axis
 *       at most: every transfer in one direction, the remark's setting); then
 *       the iterates agree with the direct form's to rounding.  With corner
 *       transfers they do not (a box's sources reach into its other overlap
 *       bands) and the iteration would lose its fixed point, so DDM_EINVAL is
 *       returned for such layouts.  On arbitrary inputs to ddm_transfer the
 *       two forms differ by beta L_a v on chi.
 * Changing the form discards captured step graphs.  DDM_EINVAL for any other
 * value. */
#define DDM_TRANSFER_DIRECT 0
#define DDM_TRANSFER_PHI 1
int ddm_set_transfer_form(ddm_handle *h, int form);

/* Library version string. */
const char *ddm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DDM_H */
