/*
 * mbs.h -- C ABI of the MI355X modified Born series (MBS) Helmholtz solver.
 *
 * Solves (nabla^2 + k^2) psi = -S on a regular 3D grid (Mache & Vellekoop,
 * arXiv 2410.02395, Sec. 2 Eq. 1) with the preconditioned Richardson iteration
 *     x <- x - alpha (I - V) (x - (L + I)^-1 [y + (I - V) x])       (Eq. 6)
 * where y = -c S, L + I is applied per subdomain as an FFT convolution
 * (Eq. 5, Sec. 3.1) and V carries the scattering potential plus the
 * truncated subdomain-communication and wrap-around-removal blocks of Sec. 3.
 * All subdomains of a plan are resident on one GPU.
 *
 * Conventions for every call:
 *   - arrays are device pointers to complex64 (interleaved float re, im),
 *     C-order [x][y][z] over the GLOBAL grid (z contiguous);
 *   - a voxel has unit size; wavenumbers are in radians per voxel;
 *   - the caller keeps ownership of every pointer it passes; the library
 *     only reads (n, S) or writes (field) them during the call, or until
 *     mbs_poll reports completion for mbs_solve_async;
 *   - the library owns all plan state (medium operator, iterate, work
 *     array, edge buffers, tables, graphs) and frees it in mbs_plan_destroy;
 *   - work is enqueued on the HIP stream given to mbs_plan_create; blocking
 *     calls synchronise that stream; a plan is used by one host thread at a
 *     time, several plans may share a device;
 *   - no exception crosses the ABI: every call returns an mbs_status.
 */
#ifndef MBS_H
#define MBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbs_plan_s* mbs_plan;
typedef int32_t mbs_status;

/* status codes (0 = success, negative = error) */
#define MBS_OK 0
#define MBS_EINVAL (-1)      /* bad shape/split/t/alpha/tol/max_iter/slot/pointer      */
#define MBS_ENOMEM (-2)      /* device allocation failed                                */
#define MBS_EGAIN (-3)       /* Im k^2 < 0 somewhere: gain medium (Sec. 2 needs a      */
                             /* passive medium for convergence)                         */
#define MBS_EDEGENERATE (-4) /* ||k^2 - k_b^2||_inf + sum_d a_d ||A12|| = 0 (Eq. 9)     */
#define MBS_ENONFINITE (-5)  /* NaN/Inf in the medium, the source or the residual       */
#define MBS_EDIVERGED (-6)   /* residual grew by more than 1 % in one iteration while   */
                             /* above 1e-5 (the iteration is monotone, Sec. 2)          */
#define MBS_ESTATE (-7)      /* solve before set_medium, or call on a busy slot         */
#define MBS_EBUSY (-8)       /* mbs_poll: the slot's solve is still running             */
#define MBS_EHIP (-9)        /* a HIP runtime call failed                               */
#define MBS_EUNSUPPORTED (-10) /* subdomain edge length outside the FFT size set         */

/* plan flags */
#define MBS_KB_FROM_K0 0x1u  /* k_b^2 = k0^2 instead of the midpoint of Re k^2          */
#define MBS_X0_GIVEN 0x2u    /* mbs_solve reads the starting field from field_dev       */
#define MBS_NO_GRAPH 0x4u    /* launch kernels one by one instead of as hipGraphs       */
#define MBS_TIMING 0x8u      /* record HIP events around every kernel kind (implies no  */
                             /* graph; the slab sequence of the strided passes as one)  */
#define MBS_NO_FUSION 0x10u  /* keep the last inverse and the next first forward z pass  */
                             /* separate (the fused pass is the default when the         */
                             /* subdomains along z fit one workgroup's line tile)        */

typedef struct {
    int64_t shape[3];    /* global grid N0, N1, N2                                          */
    int32_t split[3];    /* subdomains per axis P_d; shape[d] % split[d] == 0 (equal sizes, */
                         /* Sec. 4); subdomain edge n_d = N_d / P_d must be 2^a * 3^b with  */
                         /* b <= 1 and 8 <= n_d <= 1024                                      */
    int32_t periodic[3]; /* 1: periodic axis; 0: non-periodic (wrap-around removed, Sec. 3)  */
    int32_t t;           /* truncation of the correction blocks (Sec. 3; 8 in the paper),   */
                         /* 1 <= t <= min(16, n_d / 2) on corrected axes                     */
    int32_t max_batch;   /* number of slots (independent concurrent solves), >= 1            */
    double alpha;        /* relaxation, 0 < alpha <= 1 (0.75 in Eq. 4)                       */
    uint32_t flags;      /* MBS_* plan flags                                                 */
    int32_t check_every; /* iterations per graph launch between host checks; 0 = 16          */
    double activation;   /* subdomain activation (Sec. 3.1, end); 0 = off.  > 0: a solve     */
                         /* starts by iterating only the subdomains that hold source (all of */
                         /* them with MBS_X0_GIVEN); every check_every iterations, a         */
                         /* subdomain joins once the 2-norm of the edge terms its iterated   */
                         /* neighbours transfer into it exceeds activation * ||Gamma^-1 y||. */
                         /* Subdomains not iterated keep x = 0 and add nothing to the        */
                         /* residual; a solve that converges on the iterated set goes on if  */
                         /* some transfer still exceeds the threshold.  Needs the fused z    */
                         /* pass and at most 4096 subdomains (else MBS_EUNSUPPORTED).        */
    int32_t zblock;      /* schedule of the three strided FFT passes (y, x with the Green    */
                         /* multiply, inverse y): 0 = automatic (slabs when the work arrays  */
                         /* exceed the memory-side cache; whole subdomains alternating over  */
                         /* two streams when two fit in it), -1 = each pass over every       */
                         /* subdomain in turn, > 0 = the three passes subdomain by subdomain */
                         /* on slabs of zblock z values, so that a slab stays in the device's */
                         /* memory-side cache between them (must divide n_2 and be a         */
                         /* multiple of 16; fused z pass only, else MBS_EINVAL).  Results are */
                         /* bitwise the same either way.  With slabs, n_2 and zblock powers   */
                         /* of two and zblock < n_2, the work array is stored slab by slab    */
                         /* and the plan keeps one more complex64 array per voxel.           */
    int32_t reserved;    /* 0                                                                  */
} mbs_plan_desc;

typedef struct {
    int32_t width[3];    /* absorbing layer thickness in voxels on each side of axis d      */
    double im_n2_max;    /* Im(n^2) added at the outermost voxel; ramps linearly to 0 at the */
                         /* inner edge of the layer; the maximum over axes where they meet  */
} mbs_ramp;

typedef struct {
    int32_t iterations;  /* iterations run                                                  */
    int32_t converged;   /* 1 if rel_residual < tol                                          */
    double rel_residual; /* ||Gamma^-1 (y - A x_n)|| / ||Gamma^-1 y|| of the last iteration  */
                         /* (Sec. 3.1; one global norm over all subdomains)                  */
    double kb2;          /* k_b^2 of the splitting L = c (nabla^2 + k_b^2)                   */
    double c_imag;       /* c = i * c_imag (Eq. 9), c_imag < 0                               */
    double K;            /* ||k^2 - k_b^2||_inf                                              */
    double normC;        /* ||A12||_2 of the t x t correction block                          */
    double rho_ref;      /* ||Gamma^-1 y||                                                   */
    int32_t status;      /* MBS_OK, or the error that stopped the iteration                  */
    int64_t subdomain_iterations; /* sum over iterations of the subdomains iterated: the     */
                         /* iteration count times the subdomain count without activation   */
} mbs_result;

/* Device bytes a plan with this descriptor allocates (all slots), for HBM-budget admission
 * (Sec. 3.3 gives the paper's memory model; this plan keeps 3 complex64 arrays per voxel, 4 when
 * its slab schedule stores the work array slab by slab (zblock), plus edge buffers).  Returns
 * MBS_EINVAL/MBS_EUNSUPPORTED for descriptors mbs_plan_create rejects. */
mbs_status mbs_plan_bytes(const mbs_plan_desc* desc, size_t* device_bytes);

/* Create a plan on the current HIP device; hip_stream is a hipStream_t (NULL = default
 * stream).  Allocates everything up front; *out is NULL on error. */
mbs_status mbs_plan_create(const mbs_plan_desc* desc, void* hip_stream, mbs_plan* out);
mbs_status mbs_plan_destroy(mbs_plan plan);

/* Set the medium of a slot: k^2 = k0^2 (n^2 + i ramp) with k0 the vacuum wavenumber
 * (rad/voxel), n_dev the complex refractive index (global grid), ramp NULL for none.
 * Computes k_b^2, ||k^2 - k_b^2||_inf (FP64 reductions), c by Eq. 9 (FP64 on the host) and
 * the diagonal of (I - V).  Errors: MBS_EGAIN, MBS_ENONFINITE, MBS_EDEGENERATE. Blocking. */
mbs_status mbs_set_medium(mbs_plan plan, int32_t slot, const void* n_dev, double k0,
                          const mbs_ramp* ramp);

/* Solve for source S (src_dev, global grid).  Runs Eq. 6 from x = 0 (or from field_dev with
 * MBS_X0_GIVEN) until rel_residual < tol or max_iter iterations; tol = 0 runs exactly max_iter.
 * The residual of x_n is evaluated in iteration n; when it passes the test x_{n+1} is
 * returned.  Writes the global field to field_dev.  Not converging is not an error
 * (res->converged = 0).  Blocking. */
mbs_status mbs_solve(mbs_plan plan, int32_t slot, const void* src_dev, double tol,
                     int32_t max_iter, void* field_dev, mbs_result* res);

/* Start a solve and return at once; several slots of one plan iterate together in batched
 * launches.  mbs_poll advances the plan and returns MBS_EBUSY until the slot has finished
 * (then res, if given, holds the progress: iterations and rel_residual as of the last completed
 * launch, status MBS_EBUSY), then MBS_OK (field written, *res filled) or the solve's error. */
mbs_status mbs_solve_async(mbs_plan plan, int32_t slot, const void* src_dev, double tol,
                           int32_t max_iter, void* field_dev);
mbs_status mbs_poll(mbs_plan plan, int32_t slot, mbs_result* res);

/* Relative residual ||Gamma^-1 (y - A f)|| / ||Gamma^-1 y|| of field f (field_dev, global grid;
 * NULL = the slot's last iterate) for the slot's medium and its last source.  Costs about two
 * iterations; leaves the slot's iterate unchanged.  Blocking. */
mbs_status mbs_residual(mbs_plan plan, int32_t slot, const void* field_dev, double* rel_residual);

/* Copy the slot's per-iteration relative residuals of the last solve into host memory
 * (at most max_n values; *n receives the number written). */
mbs_status mbs_residual_history(mbs_plan plan, int32_t slot, double* host_out, int32_t max_n,
                                int32_t* n);

/* Kernel timing (plans created with MBS_TIMING): per kernel kind, the summed HIP-event
 * duration in ms and the launch count since the last reset.  Kinds, in order:
 * 0 forward pass (z), 1 forward pass (y), 2 Green pass (x), 3 inverse pass (y),
 * 4 inverse pass with update (z), 5 edge corrections, 6 face update, 7 residual
 * reduction.  With the fused z pass, kind 4 also forms the next w and its forward z FFT,
 * kind 0 covers only the lines of the x/y edge slabs and kind 6 finishes those lines.
 * Kind 8: kinds 1-3 run slab by slab (mbs_plan_desc.zblock), timed as one.  n_kinds <= 9. */
mbs_status mbs_timing_read(mbs_plan plan, double* ms, int64_t* launches, int32_t n_kinds,
                           int32_t reset);

const char* mbs_strerror(mbs_status status);

#ifdef __cplusplus
}
#endif

#endif /* MBS_H */
