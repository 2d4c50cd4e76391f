/*
 * numag.h -- C ABI of the MI355X (gfx950) direct-Fourier-sum SANS library.
 *
 * The library computes the nuclear and magnetic small-angle neutron
 * scattering observables of NuMagSANS (Adams & Michels, arXiv 2601.18444)
 * from user-given point data: nuclear scattering lengths n_j and magnetic
 * moments m_j at positions x_j of K objects with offsets r^k, after a sample
 * rotation R, on a 2D detector in the y-z plane (beam along x).
 *
 * Conventions (each is the library's reading of the paper):
 *   - Sums are raw:  S_c(q) = sum_j w_{j,c} exp(-i q . X_j),  c = N, Mx, My, Mz,
 *     with X_j = R (x_j + r^{k(j)}) (Sec. 3.2 position transform),
 *     w_{j,N} = n_j and (w_{j,Mx}, w_{j,My}, w_{j,Mz}) = R m_j (moments turn with
 *     the sample, as the alpha = 90 deg example of Sec. 3.1 requires), and
 *     q = (0, q_y, q_z) (Sec. 2.1 eq. qdef).  The DSFT prefactor (2 pi)^{-3/2}
 *     and the 8 pi^3 of the cross sections cancel, and the (W Nbar)^{-1/2}
 *     normalisation of Sec. 3.3 is undone by its absolute-unit rescale, so
 *     every cross section is (scale / V) times a quadratic form in S.
 *   - Halpern-Johnson vector Q = qhat x (qhat x M) (eq. HJdef) for every
 *     signed term.
 *   - Cartesian detector: q_i = -qmax + i * (2 qmax / (n - 1)) (FP64, one product
 *     and one sum, no fused multiply-add); pixel p = i_y * n_z + i_z; the q = 0
 *     pixel (odd n only) takes qhat = e_z.
 *   - Polar detector (the paper's (q, theta) grid, Sec. 3.1/3.2):
 *     q_i = i * qmax / (n_q - 1), theta_m = 2 pi m / n_theta,
 *     q_y = q sin(theta), q_z = q cos(theta); pixel p = i_q * n_theta + m.
 *   - Complex numbers are two doubles (re, im).
 *
 * Memory: every array argument is DEVICE memory owned by the caller unless the
 * comment says "host".  The library never frees caller memory.  All work is
 * enqueued on `stream` (a hipStream_t; NULL is the null stream) and returns
 * before it completes.  Every entry point validates all arguments before any
 * work is enqueued; an invalid call returns a negative status, enqueues
 * nothing and leaves a message for numag_last_error() (per thread).
 *
 * Tuning: launch shapes come from a table (numag_tune_get / numag_autotune
 * below); without an entry, the environment variable NUMAG_TARGET_WGS (read
 * once per process) sets the number of workgroups the direct sums aim for per
 * launch (default 2048, the value measured best on MI355X; the polar sums take
 * half, the adjoint twice).  Shapes change how the work is split, never a
 * result's definition; sums split differently agree to rounding.
 */
#ifndef NUMAG_H
#define NUMAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define NUMAG_OK             0
#define NUMAG_E_INVALID     -1  /* a bad argument; nothing was enqueued          */
#define NUMAG_E_WORKSPACE   -2  /* workspace too small; nothing was enqueued     */
#define NUMAG_E_HIP         -4  /* a HIP runtime call failed                     */
#define NUMAG_E_UNSUPPORTED -5  /* valid request the library does not implement  */

/* ---- detector kinds ----------------------------------------------------- */
#define NUMAG_GRID_CARTESIAN 0
#define NUMAG_GRID_POLAR     1

/* ---- summation paths ---------------------------------------------------- */
/* Direct sum over points (any point cloud, any rotation, Cartesian or polar
   detector), FP64 accumulation; the general path. */
#define NUMAG_PATH_DIRECT         0
/* Regular-grid separable path: requires sample->regular, R = identity, one
   object and a Cartesian detector.  The sum over x is a projection and the
   rest is two dense complex contractions on the matrix cores. */
#define NUMAG_PATH_SEPARABLE_F64  1  /* FP64 matrix-core contractions        */
/* BF16 split products on the matrix cores (FP32 accumulation): every operand
   split into 2 (X3: 3 products per real product) or 3 (X6: 6 products) bf16
   parts.  Measured on the 64^3 vortex grid (256 x 256 detector) against the
   FP64 path, gated relative error of the 13 cross sections: X3 8e-4 .. 2e-2,
   X6 9e-6 .. 7e-5 except 2.6e-4 on the nuclear-magnetic interference.  Neither
   meets the 1e-4 gate of the matrix-core path on every observable; they are
   provided for speed comparisons. */
#define NUMAG_PATH_SEPARABLE_BF16X3 2
/* Direct path on half of a detector that is symmetric about q = 0 (every
   Cartesian detector; a polar one with an even n_theta), the other half filled
   by S(-q) = conj S(q), which holds because the weights are real: half the
   work, the same sums up to rounding (the mirrored pixel takes the conjugate
   of its partner's sum instead of a sum over its own q, which differs from -q
   by at most an ulp).  All modes: in DILUTE / SPLIT the spectral matrices
   follow G(-q) = conj G(q) and the coherent total A(-q) = conj A(q), for
   every rotation. */
#define NUMAG_PATH_DIRECT_HERMITIAN 3
#define NUMAG_PATH_SEPARABLE_BF16X6 4  /* see NUMAG_PATH_SEPARABLE_BF16X3 */
/* FP64 separable path on half of the (symmetric) Cartesian detector: the second
   contraction runs on rows [0, ceil(n0 / 2)) only and writes each pixel's
   conjugate at the mirrored pixel, S(-q) = conj S(q) for real weights -- half of
   the dominant contraction's work.  The computed rows equal the full path's bit
   for bit; a mirrored pixel takes its partner's conjugate instead of a sum over
   its own q (which differs from -q by at most an ulp).  Same arguments,
   workspace and outputs as NUMAG_PATH_SEPARABLE_F64. */
#define NUMAG_PATH_SEPARABLE_F64_HERMITIAN 5

/* ---- object modes (Sec. 3.3, summation relation and dilute limit) -------- */
#define NUMAG_MODE_COHERENT 0  /* |sum_k exp(-i q.R r^k) F_k|^2                   */
#define NUMAG_MODE_DILUTE   1  /* sum_k |F_k|^2  (no StructData: r^k unused)      */
#define NUMAG_MODE_SPLIT    2  /* both: coherent total and the form-factor part   */

/* ---- observables (bit index = order of output rows) ---------------------- */
#define NUMAG_OBS_N      (1u << 0)   /* eq. NuclearSANS                            */
#define NUMAG_OBS_M      (1u << 1)   /* eq. MagneticSANS                           */
#define NUMAG_OBS_NM     (1u << 2)   /* eq. NMdef, nuclear-magnetic interference   */
#define NUMAG_OBS_P      (1u << 3)   /* eq. PSANSdef                               */
#define NUMAG_OBS_CHI    (1u << 4)   /* eq. ChiralSANS, the real dSigma_chi        */
#define NUMAG_OBS_SF     (1u << 5)   /* eq. sfdef, spin-flip M - P                 */
#define NUMAG_OBS_PP     (1u << 6)   /* ++ = N + NM + P           (Sec. 2.2)       */
#define NUMAG_OBS_MM     (1u << 7)   /* -- = N - NM + P                            */
#define NUMAG_OBS_PM     (1u << 8)   /* +- = SF + CHI                              */
#define NUMAG_OBS_MP     (1u << 9)   /* -+ = SF - CHI                              */
#define NUMAG_OBS_PLUS   (1u << 10)  /* SANSPOL + = ++ + +-       (Sec. 2.3)       */
#define NUMAG_OBS_MINUS  (1u << 11)  /* SANSPOL - = -- + -+                        */
#define NUMAG_OBS_UNPOL  (1u << 12)  /* unpolarized (++ + -- + +- + -+)/2 (Sec. 2.4) */
#define NUMAG_OBS_ALL    0x1FFFu

/* A regular grid of points (micromagnetic cells): point j = (ix * ny + iy) * nz + iz
   sits at origin + (ix, iy, iz) * step.  Host struct. */
typedef struct {
    int32_t n[3];
    int32_t reserved;
    double origin[3];
    double step[3];
} numag_regular;

/* Real-space input (Sec. 3.2: NucData, MagData, StructData). */
typedef struct {
    int64_t n_points;             /* W >= 0                                           */
    const double *pos;            /* [W][3] local coordinates x^{kl} (nm); may be NULL
                                     only when `regular` is given                      */
    const double *nuc;            /* [W] nuclear scattering lengths, or NULL (channel off) */
    const double *mag;            /* [W][3] magnetic moments, or NULL (channel off)    */
    int64_t n_objects;            /* K >= 1                                           */
    const int64_t *obj_offsets;   /* HOST [K+1] CSR offsets (obj k = points off[k] ..
                                     off[k+1]-1, off[0] = 0, off[K] = W); NULL iff K = 1 */
    const double *obj_pos;        /* [K][3] object positions r^k (nm), or NULL (= 0)    */
    const numag_regular *regular; /* HOST, or NULL: points form this regular grid       */
} numag_sample;

/* Detector (Sec. 3.1: q_max and resolutions).  Host struct. */
typedef struct {
    int32_t kind;                 /* NUMAG_GRID_CARTESIAN or NUMAG_GRID_POLAR          */
    int32_t n0;                   /* Cartesian: n_y (rows);  polar: n_q  (rows)       */
    int32_t n1;                   /* Cartesian: n_z (cols);  polar: n_theta (cols)    */
    int32_t reserved;
    double qmax;                  /* nm^-1, > 0                                        */
} numag_qgrid;

/* Constants of the cross sections (Sec. 2.1, Sec. 3.3 absolute-unit rescale).
   Every observable is (scale / V) times its quadratic form, with one factor bH
   per magnetic amplitude.  Host struct. */
typedef struct {
    double V;                     /* scattering volume, > 0                             */
    double bH;                    /* magnetic scattering length (2.91e8 A^-1 m^-1 in SI) */
    double scale;                 /* unit factor (e.g. 1e-2 for m^-1 -> cm^-1)           */
    double P[3];                  /* polarisation unit vector Phat                      */
} numag_consts;

/*
 * Workspace bytes numag_amplitudes / numag_grad need for this request
 * (0 when none).  Returns 0 and sets numag_last_error() on invalid input.
 */
size_t numag_workspace_size(const numag_sample *sample, int64_t n_rot, const numag_qgrid *grid,
                            int32_t path, int32_t mode);

/*
 * Direct Fourier sums, Sec. 3.3 (DSFT and its cos/sin split), per object mode
 * (Sec. 3.3 summation relation and dilute approximation), for n_rot sample
 * rotations (Sec. 3.1; any R in SO(3)).
 *   rot       HOST [n_rot][9] row-major rotation matrices, or NULL (identity;
 *             then n_rot must be 1).  Each must be orthonormal with det +1
 *             (|R R^T - I| <= 1e-9), else NUMAG_E_INVALID.
 *   amp_out   [n_rot][P][4] complex (COHERENT, SPLIT): the coherent sums
 *             S_c = sum_k exp(-i q.R r^k) F_k; NULL in DILUTE mode.
 *   spec_out  [n_spec][P][16] (DILUTE, SPLIT): the spectral matrix
 *             G_ab = (1/n_rot) sum_rot sum_k F_{k,a} conj(F_{k,b}) packed as
 *             [G00 G11 G22 G33, Re G01, Im G01, Re G02, Im G02, Re G03, Im G03,
 *              Re G12, Im G12, Re G13, Im G13, Re G23, Im G23]; n_spec = K when
 *             spec_per_object != 0 (one matrix per object, averaged over the
 *             rotations), else 1 (summed over objects).  NULL in COHERENT mode.
 *   path      NUMAG_PATH_*; the separable paths need sample->regular, rot NULL,
 *             K = 1, a Cartesian detector and COHERENT mode;
 *             NUMAG_PATH_DIRECT_HERMITIAN needs an even n_theta on a polar
 *             detector.
 *   mode      DILUTE and SPLIT need explicit positions (NUMAG_E_UNSUPPORTED for
 *             a regular-grid sample); SPLIT takes one rotation.  Both run on
 *             either detector kind as one persistent launch over (object group,
 *             rotation range, pixel block) work items.  These
 *             modes build a one-off plan (see numag_plan_create) on every call:
 *             its tables (object offsets, rotations, work items) are copied to
 *             the start of the workspace from host memory the library frees
 *             once the stream has passed the copy; the call never waits for the
 *             stream.  Such a call cannot be captured into a graph
 *             (NUMAG_E_UNSUPPORTED while `stream` is capturing): capture
 *             numag_amplitudes_plan instead.
 *   workspace device scratch of at least numag_workspace_size() bytes; its
 *             contents are undefined after the call.
 * COHERENT mode copies nothing from the host (it enqueues kernels only).
 * Empty samples (W = 0) are valid and give zeros.
 */
int numag_amplitudes(const numag_sample *sample, int64_t n_rot, const double *rot,
                     const numag_qgrid *grid, int32_t path, int32_t mode, int32_t spec_per_object,
                     double *amp_out, double *spec_out, void *workspace, size_t ws_bytes,
                     void *stream);

/*
 * Allocation-free coherent sums, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): numag_amplitudes in COHERENT mode on NUMAG_PATH_DIRECT or
 * NUMAG_PATH_DIRECT_HERMITIAN, same arguments and outputs (amp_out [n_rot][P][4]
 * complex, device) but no workspace.
 *   Scratch: the point records and split partial sums live in one static device
 *   array of NUMAG_NOALLOC_SCRATCH_BYTES that the library holds on every device
 *   it runs on until the process ends; its device address is looked up on the
 *   first call on a device.  Points go through in chunks, so any W fits; the
 *   partial sums of the evaluated pixels (64 bytes each: the whole detector, or
 *   the half that the Hermitian path sums) must fit in half of the array, at
 *   most 1,048,576 evaluated pixels, else NUMAG_E_UNSUPPORTED with a message.
 *   Calls on one device share the array: calls that may overlap in time on one
 *   device (streams not ordered with each other, or other host threads) race
 *   and give wrong results; calls ordered on one stream are safe.  Nothing in
 *   the array has to start at zero (a call writes every byte it reads).
 *   The call enqueues kernels only: no hipMalloc, hipFree or host-to-device
 *   copy, and no wait for the stream (with the kernel timer disabled, since it
 *   creates events on demand).  The sums equal numag_amplitudes' up to rounding
 *   (the points may be split differently).
 */
#define NUMAG_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int numag_amplitudes_noalloc(const numag_sample *sample, int64_t n_rot, const double *rot,
                             const numag_qgrid *grid, int32_t path, double *amp_out, void *stream);

/*
 * Object-mode plans (Sec. 3.3 summation relation and dilute limit, for many
 * sample rotations): the host-side part of a DILUTE or SPLIT request -- object
 * offsets, rotations and, on a Cartesian detector, the persistent kernel's
 * work items -- built once, uploaded once into a caller workspace, then used
 * by any number of numag_amplitudes_plan calls that enqueue kernels only (so
 * they can be recorded into a HIP graph and replayed).
 *   numag_plan_create   validates as numag_amplitudes does (mode DILUTE or
 *             SPLIT, path DIRECT or DIRECT_HERMITIAN) and copies what it needs
 *             of the host arguments (rot HOST [n_rot][9] or NULL, the sample's
 *             HOST object offsets); *plan_out receives the handle.
 *   numag_plan_workspace_size   bytes of the workspace the plan's calls need.
 *   numag_plan_upload   enqueues the copy of the plan's tables (held in host
 *             memory owned by the plan) to the start of `workspace`: the plan
 *             must not be destroyed before the stream has passed that copy.
 *   numag_amplitudes_plan   the sums of the plan for `sample`, whose point
 *             count, object count and object offsets must equal the plan's (its
 *             device arrays -- positions, weights, object positions -- may
 *             differ from call to call).  The workspace must hold the plan's
 *             upload: only its tables region (the start of the workspace) must be
 *             left untouched between calls; the rest is scratch.  Every table read
 *             is guarded by a tag unique to the plan, written at the start of its
 *             upload: a workspace that does not hold this plan's upload (never
 *             uploaded, overwritten, or another buffer) gives NaN outputs instead
 *             of reading foreign tables.  Outputs as numag_amplitudes (amp_out
 *             only in SPLIT mode).
 *   numag_plan_destroy  frees the handle (NULL is a no-op).
 */
typedef struct numag_plan numag_plan;
int numag_plan_create(const numag_sample *sample, int64_t n_rot, const double *rot, const numag_qgrid *grid,
                      int32_t path, int32_t mode, int32_t spec_per_object, numag_plan **plan_out);
size_t numag_plan_workspace_size(const numag_plan *plan);
int numag_plan_upload(const numag_plan *plan, void *workspace, size_t ws_bytes, void *stream);
int numag_amplitudes_plan(const numag_plan *plan, const numag_sample *sample, double *amp_out, double *spec_out,
                          void *workspace, size_t ws_bytes, void *stream);
void numag_plan_destroy(numag_plan *plan);

/*
 * Loop mode (Sec. 3.1 loop modes; Sec. 3.2: one real-space data set per field,
 * temperature or time value): the raw sums of n_snap weight snapshots given on
 * one regular grid, unrotated, one object, on a Cartesian detector, by a
 * separable path (NUMAG_PATH_SEPARABLE_F64, _F64_HERMITIAN, _BF16X3 or _BF16X6) in
 * one batched call.
 *   points    HOST regular grid of the W = n[0] n[1] n[2] points (as numag_sample.regular)
 *   nuc       [n_snap][W] or NULL (channel off);  mag [n_snap][W][3] or NULL
 *   amp_out   [n_snap][P][4] complex: snapshot b equals numag_amplitudes of
 *             snapshot b alone on the same path.
 *   workspace at least numag_snapshots_workspace_size() bytes (it grows with
 *             n_snap: 4 n_snap (ny nz + 2 ny n1) doubles plus the twiddles, each
 *             dimension padded to the matrix-core tiles).
 * Returns NUMAG_E_INVALID for n_snap < 1, a non-separable path, a polar
 * detector or a bad grid; numag_snapshots_workspace_size returns 0 then.
 */
size_t numag_snapshots_workspace_size(const numag_regular *points, int64_t n_snap, const numag_qgrid *grid,
                                      int32_t path);
int numag_amplitudes_snapshots(const numag_regular *points, int64_t n_snap, const double *nuc, const double *mag,
                               const numag_qgrid *grid, int32_t path, double *amp_out, void *workspace,
                               size_t ws_bytes, void *stream);

/*
 * Cross sections of Sec. 2 (eqs. NuclearSANS, MagneticSANS, HJdef, PSANSdef,
 * sfdef, ChiralSANS, NMdef; the POLARIS, SANSPOL and unpolarized combinations
 * of Sec. 2.2-2.4) from n_sets amplitude sets or spectral matrices.
 *   amp       [n_sets][P][4] complex, or NULL
 *   spec      [n_sets][P][16] packed spectral matrices (as numag_amplitudes
 *             writes them), or NULL; exactly one of amp/spec is given.
 *   obs_mask  NUMAG_OBS_* bits; rows of `out` follow increasing bit order.
 *   out       [n_sets][popcount(obs_mask)][P] doubles.
 * With n_sets = 0 nothing is written and amp, spec and out may all be NULL.
 */
int numag_cross_section(const numag_qgrid *grid, int64_t n_sets, const double *amp,
                        const double *spec, const numag_consts *consts, uint32_t obs_mask,
                        double *out, void *stream);

/*
 * Export of the Fourier cross-correlation functions (Sec. 3.4: G^R_ab = Re,
 * G^I_ab = Im of M_a conj(M_b)), extended by the nuclear channel: for every
 * amplitude set and pixel, G_ab = A_a conj(A_b) over a, b in (N, Mx, My, Mz),
 * packed as numag_amplitudes packs spectral matrices (16 reals: the four
 * diagonal entries, then Re/Im of the upper entries 01 02 03 12 13 23).  Any
 * detector kind.  No unit factors are applied.
 *   amp       [n_sets][P][4] complex (device);  spec_out [n_sets][P][16] (device)
 */
int numag_spectral_matrix(const numag_qgrid *grid, int64_t n_sets, const double *amp, double *spec_out,
                          void *stream);

/*
 * Azimuthal average, eq. iqazi, for n_f 2D data sets f [n_f][P].
 * Cartesian detector: equal-width annuli of [0, qmax_avg] (bin b holds
 *   b*dq <= |q| < (b+1)*dq with dq = qmax_avg / n_bins, |q| = qmax_avg in the last
 *   bin, |q| > qmax_avg dropped); value = mean of the bin; empty bins are NaN.
 *   Bin centres are (b + 1/2) dq.
 * Polar detector: the periodic trapezoidal rule over theta of every q row;
 *   n_bins must equal n_q and qmax_avg is ignored.
 *   I_out     [n_f][n_bins];  count_out [n_bins] int64 or NULL.
 * With n_f = 0 nothing is written, count_out included.
 */
int numag_azimuthal_average(const numag_qgrid *grid, const double *f, int32_t n_f, int32_t n_bins,
                            double qmax_avg, double *I_out, int64_t *count_out, void *stream);

/*
 * Correlation and pair-distance distribution functions, eqs. crrad and prrad:
 *   c(r) = (scale / 2 pi^2) int I(q) j0(q r) q^2 dq,   p(r) = r^2 c(r),
 * by the trapezoidal rule over the nodes (0, 0) and (q_b, I_b q_b^2 j0(q_b r));
 * NaN samples of I are skipped.  scale = 1 is eq. crrad as printed; the
 * p_max values of the paper's Tables I and II correspond to scale = 2 pi^2.
 *   q [n_q] ascending, I [n_f][n_q], r [n_r];  c_out, p_out [n_f][n_r].
 */
int numag_correlation(const double *q, const double *I, int32_t n_q, int32_t n_f, const double *r,
                      int32_t n_r, double scale, double *c_out, double *p_out, void *stream);

/*
 * Loss on the unpolarized cross section (Sec. 2.4) and its gradient with
 * respect to every input weight (the adjoint, i.e. transposed, Fourier sum):
 *   I_p = (scale/V)(|S_N|^2 + bH^2 |Q|^2),   L = sum_p w_p (I_p - T_p)^2,
 *   dL/dn_j and dL/dm_j (the unrotated input moments: R^T dL/dm'_j).
 * One rotation (rot HOST [9] or NULL), COHERENT mode, direct path.
 *   amp_in    [P][4] complex sums of this sample (as numag_amplitudes writes
 *             them), or NULL to compute them here.
 *   target, weight  [P];  loss_out  [1] double (device).
 *   target NULL: `weight` holds an upstream gradient dL/dI_p instead (the
 *             backward of an autograd function) and loss_out may be NULL;
 *   dnuc_out  [W] or NULL;  dmag_out [W][3] or NULL.
 *   workspace of at least numag_workspace_size(sample, 1, grid, path,
 *             NUMAG_MODE_COHERENT) bytes.
 * numag_grad is numag_grad_path with NUMAG_PATH_DIRECT.  With
 * NUMAG_PATH_DIRECT_HERMITIAN (a polar detector needs an even n_theta) the
 * sums (when amp_in is NULL) and the adjoint run on half of the detector: the
 * residual weight of each pixel's mirror p' (at -q within an ulp) is folded
 * onto it as a(p) + conj a(p'), since Re[a(p') exp(+i q.X)] =
 * Re[conj a(p') exp(-i q.X)]; this holds for any target and loss weights.  The
 * loss is evaluated over the whole detector.
 */
int numag_grad(const numag_sample *sample, const double *rot, const numag_qgrid *grid,
               const numag_consts *consts, const double *amp_in, const double *target,
               const double *weight, double *loss_out, double *dnuc_out, double *dmag_out,
               void *workspace, size_t ws_bytes, void *stream);
int numag_grad_path(const numag_sample *sample, const double *rot, const numag_qgrid *grid, int32_t path,
                    const numag_consts *consts, const double *amp_in, const double *target,
                    const double *weight, double *loss_out, double *dnuc_out, double *dmag_out,
                    void *workspace, size_t ws_bytes, void *stream);

/*
 * Two-dimensional correlation function, eq. crav2d,
 *   C(rho, alpha) = int int f(q, theta) exp(i q rho cos(theta - alpha)) q dq dtheta,
 * evaluated as the trapezoidal quadrature over the detector `grid` (polar:
 * weights h_i q_i dtheta with h_i = dq halved at q = 0 and q_max; Cartesian:
 * dq_y dq_z with halved edge rows/columns) at the points of the real-space grid
 * `rgrid` (same descriptor; its qmax is r_max in nm: Cartesian r on [-r_max, r_max]^2,
 * polar rho_a = a r_max / (n_rho - 1), alpha_b = 2 pi b / n_alpha with
 * r = rho (sin alpha, cos alpha)).
 *   f       [n_f][P] data sets on `grid`
 *   C_out   [n_f][R][2] complex (R = rgrid pixels)
 *   workspace of at least numag_correlation_2d_workspace_size() bytes.
 */
size_t numag_correlation_2d_workspace_size(const numag_qgrid *grid, const numag_qgrid *rgrid);
int numag_correlation_2d(const numag_qgrid *grid, const double *f, int32_t n_f, const numag_qgrid *rgrid,
                         double *C_out, void *workspace, size_t ws_bytes, void *stream);

/*
 * Angular spectrum, eqs. CosineSinceIntensities and ModalAmplitudes, on a polar
 * detector (periodic trapezoidal rule over theta):
 *   I_k^{s,c}(q_i) = (2 - delta_k0)/(2 pi) int f(q_i, theta) {sin, cos}(k theta) dtheta,
 *   a_k = sum_i I_k(q_i),  A_k = a_k / sum_j sqrt(a_j^s^2 + a_j^c^2),  0 <= k <= k_max.
 *   Is_out, Ic_out [n_f][n_q][k_max+1];  As_out, Ac_out [n_f][k_max+1] or NULL.
 */
int numag_angular_spectrum(const numag_qgrid *grid, const double *f, int32_t n_f, int32_t k_max, double *Is_out,
                           double *Ic_out, double *As_out, double *Ac_out, void *stream);

/*
 * Launch shapes and their autotuner (the paper's runtime scales over three
 * decades of point counts, Sec. 4.4, so no single launch shape suits every
 * workload).  A shape cuts a kernel's work into workgroups and point splits; it
 * never changes what is summed, so sums under different shapes agree to
 * rounding.  Shapes are kept in a process-wide table keyed by (kernel, detector
 * kind and the size of the part a path evaluates, the point count's half-octave
 * class floor(2 log2 W), GPU architecture); a kernel without an entry uses the
 * library default.  With NUMAG_AUTOTUNE_CACHE naming a file, the table is read
 * from it on the first lookup and rewritten after every numag_autotune (one
 * text line per entry).
 *   kernel    NUMAG_TUNE_DIRECT (direct sums; the detector kind selects the
 *             Cartesian or the polar kernel), NUMAG_TUNE_ADJOINT (the gradient's
 *             adjoint sums), NUMAG_TUNE_OBJECTS (the persistent object kernel of
 *             DILUTE / SPLIT modes on a Cartesian detector).
 *   shape     Cartesian direct and objects: lanes per detector row (8, 16, 32,
 *             64); polar direct: workgroup shape 0-4 (0: 64 q rows x 64 theta
 *             columns; 1: 32 x 64, only for at most 32 q rows; 2: 128 x 32;
 *             3: 256 x 16 with chunks of 16 points; 4: 256 x 16 with
 *             double-buffered chunks of 8 points); adjoint: 0.
 *   target    workgroups a launch aims for (objects: work items); 0 = default.
 *   path      NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN (which part of
 *             the detector is evaluated).
 * numag_tune_get writes the default and the shape in use (either pointer may be
 * NULL) and returns 1 if the table holds an entry in use, 0 if the default is
 * used, or a negative status.  numag_tune_set stores a shape (NULL removes the
 * entry; NUMAG_E_INVALID for a shape the kernel cannot take on this detector).
 * numag_autotune times the candidate shapes of `kernel` on the caller's sample
 * and detector (the direct and adjoint kernels on the first max_points points
 * as one object when max_points > 0; the object kernel on the first 64 of the
 * rotations, all objects), keeps the fastest in the table (the default unless
 * another is more than 1 % faster), writes it to *chosen_out (may be NULL) and
 * saves the cache file if one is named.  It allocates its own trial buffers,
 * waits for the stream and cannot run under graph capture; call it when no
 * other call of this library is in flight (workspace sizes follow the table:
 * query them again after tuning).
 */
typedef struct {
    int32_t shape;
    int32_t target;
} numag_tune_shape;
#define NUMAG_TUNE_DIRECT  0
#define NUMAG_TUNE_ADJOINT 1
#define NUMAG_TUNE_OBJECTS 2
int numag_tune_get(int32_t kernel, const numag_qgrid *grid, int32_t path, int64_t n_points,
                   numag_tune_shape *default_out, numag_tune_shape *current_out);
int numag_tune_set(int32_t kernel, const numag_qgrid *grid, int32_t path, int64_t n_points,
                   const numag_tune_shape *shape);
int numag_tune_clear(void);
int numag_autotune(const numag_sample *sample, int64_t n_rot, const double *rot, const numag_qgrid *grid,
                   int32_t path, int32_t kernel, int64_t max_points, numag_tune_shape *chosen_out, void *stream);

/*
 * Kernel timer, for measurement harnesses.  While enabled, the library records
 * a HIP event pair on the caller's stream around every launch of its sum
 * kernels (the events are enqueued like the kernels: nothing blocks).  Leave
 * it disabled while a stream is being captured into a graph.
 *   numag_kernel_timer(1) enables and clears, numag_kernel_timer(0) disables
 *   (the recorded launches stay readable).
 *   numag_kernel_timer_read waits for the recorded launches of `kernel`
 *   (NUMAG_KERNEL_*), writes their summed duration in milliseconds and their
 *   count (either pointer may be NULL) and forgets them.
 * Returns NUMAG_OK, NUMAG_E_INVALID for an unknown kernel id, or NUMAG_E_HIP.
 */
#define NUMAG_KERNEL_DIRECT   0  /* Cartesian or polar direct sum kernel   */
#define NUMAG_KERNEL_ADJOINT  1  /* adjoint (gradient) sum kernel          */
#define NUMAG_KERNEL_OBJECTS  2  /* object/orientation work-queue kernel   */
#define NUMAG_KERNEL_COUNT    3
int numag_kernel_timer(int32_t enable);
int numag_kernel_timer_read(int32_t kernel, double *total_ms, int64_t *launches);

/* Message of the last failing call on this thread ("" if none). */
const char *numag_last_error(void);

/* Library version string. */
const char *numag_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NUMAG_H */
