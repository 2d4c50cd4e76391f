/*
 * numag oracle: a plain, slow FP64 CPU implementation of the direct-Fourier-sum
 * SANS path of NuMagSANS (Adams & Michels, arXiv 2601.18444).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load, call or execute this library.  It
 * shares no code, header, table or helper with the HIP path, and the HIP path
 * never calls it.
 *
 * Every routine is the paper's definition written out with no blocking, fusion
 * or reordering: double loops in FP64 with libm sin/cos, OpenMP only over
 * independent output elements.  Complex arithmetic uses C99 complex.
 *
 * Conventions frozen here (each is a reading of the paper):
 *   - sums are the raw discrete sums S(q) = sum_j w_j exp(-i q.r_j); the
 *     (2 pi)^{-3/2} of the DSFT and the 8 pi^3 of the cross sections cancel
 *     (Sec. 2.1 eqs. NuclearSANS/MagneticSANS with Sec. 3.3), and the
 *     (W Nbar)^{-1/2} normalisation is undone by the absolute-unit rescale
 *     (Sec. 3.3), so every cross section is (scale/V) times a quadratic form
 *     in the raw sums;
 *   - positions are X = R (x + r^k) (Sec. 3.2) and moments rotate with the
 *     sample, m' = R m (Sec. 3.1, the alpha = 90 deg example);
 *   - the lab scattering vector is q = (0, q_y, q_z) (Sec. 2.1, eq. qdef);
 *   - the unit vector qhat is given per pixel by the caller (the q = 0 pixel
 *     has no direction; its reading is the caller's);
 *   - Q = qhat x (qhat x M) (eq. HJdef), used for every signed term.
 *
 * Parity status: every function here is pinned by tests under tests/ that
 * do not call it to make their expected values (closed forms, brute force,
 * identities); see the header of each function.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Geometry: Sec. 3.2, position transform with object offsets.               */
/* R is row-major: R[3*a + b] = R_{a+1, b+1}.                                 */
/* ------------------------------------------------------------------------ */
static void mat_vec(const double *R, const double v[3], double out[3])
{
    for (int a = 0; a < 3; ++a)
        out[a] = R[3 * a + 0] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2];
}

/* Object index of every point from the CSR offsets (object k owns points
   off[k] .. off[k+1]-1); all zero for a single object.  Caller frees. */
static int64_t *object_index(int64_t W, int64_t K, const int64_t *off)
{
    int64_t *kidx = (int64_t *)calloc((size_t)(W > 0 ? W : 1), sizeof(int64_t));
    if (K > 1 && off != NULL)
        for (int64_t k = 0; k < K; ++k)
            for (int64_t j = off[k]; j < off[k + 1]; ++j) kidx[j] = k;
    return kidx;
}

/*
 * Discrete Fourier sums of Sec. 3.3 (the DSFT, and its cos/sin split):
 *   A[p][c] = sum_j w_{j,c} exp(-i q_p . X_j),  c in {N, Mx, My, Mz},
 * with w_{j,N} = nuc[j] and (w_{j,Mx}, w_{j,My}, w_{j,Mz}) = R mag[j], and
 * X_j = R (x_j + r^{k(j)}) (Sec. 3.2).  q_p = (0, qy[p], qz[p]).
 *
 * per_object == 0: coherent total, out is [n_pix][4] complex.
 * per_object == 1: the object amplitudes F_k of Sec. 3.3 (summation relation
 *   and the dilute approximation), out is [K][n_pix][4] complex, computed
 *   from the local coordinates x^{kl} only (r^k dropped).
 * nuc or mag may be NULL (that channel is zero).
 */
void orc_amplitudes(int64_t W, const double *pos, const double *nuc, const double *mag,
                    int64_t K, const int64_t *off, const double *obj_pos,
                    const double *R, int64_t n_pix, const double *qy, const double *qz,
                    int per_object, double *out_ri)
{
    cplx *out = (cplx *)out_ri;
    int64_t n_sets = per_object ? (K > 0 ? K : 1) : 1;
    memset(out_ri, 0, sizeof(cplx) * (size_t)(n_sets * n_pix * 4));
    int64_t *kidx = object_index(W, K, off);

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < n_pix; ++p) {
        for (int64_t j = 0; j < W; ++j) {
            int64_t k = kidx[j];
            double x[3] = {pos[3 * j + 0], pos[3 * j + 1], pos[3 * j + 2]};
            if (!per_object && obj_pos != NULL) {
                x[0] += obj_pos[3 * k + 0];
                x[1] += obj_pos[3 * k + 1];
                x[2] += obj_pos[3 * k + 2];
            }
            double X[3];
            mat_vec(R, x, X);
            double m[3] = {0.0, 0.0, 0.0}, mr[3] = {0.0, 0.0, 0.0};
            if (mag != NULL) {
                m[0] = mag[3 * j + 0];
                m[1] = mag[3 * j + 1];
                m[2] = mag[3 * j + 2];
                mat_vec(R, m, mr);
            }
            double n = (nuc != NULL) ? nuc[j] : 0.0;
            /* phase function Psi = q (Y sin(theta) + Z cos(theta)) = qy Y + qz Z */
            double psi = qy[p] * X[1] + qz[p] * X[2];
            cplx e = cos(psi) - I * sin(psi);
            cplx *dst = out + ((per_object ? k : 0) * n_pix + p) * 4;
            dst[0] += n * e;
            dst[1] += mr[0] * e;
            dst[2] += mr[1] * e;
            dst[3] += mr[2] * e;
        }
    }
    free(kidx);
}

/*
 * Spectral (cross-correlation) matrix of Sec. 3.4 extended by the nuclear
 * channel: G_ab(q) = sum_s A_{s,a}(q) conj(A_{s,b}(q)), summed over the n_sets
 * amplitude sets given (objects of a dilute sample, rotations, ...).
 * Output per pixel: 16 reals [G00 G11 G22 G33, Re G01, Im G01, Re G02, Im G02,
 * Re G03, Im G03, Re G12, Im G12, Re G13, Im G13, Re G23, Im G23].
 */
void orc_spectral(int64_t n_sets, int64_t n_pix, const double *amp_ri, double *G)
{
    const cplx *A = (const cplx *)amp_ri;
    static const int pa[6] = {0, 0, 0, 1, 1, 2};
    static const int pb[6] = {1, 2, 3, 2, 3, 3};
#pragma omp parallel for
    for (int64_t p = 0; p < n_pix; ++p) {
        cplx g[4][4];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) g[a][b] = 0.0;
        for (int64_t s = 0; s < n_sets; ++s) {
            const cplx *v = A + (s * n_pix + p) * 4;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) g[a][b] += v[a] * conj(v[b]);
        }
        double *o = G + p * 16;
        for (int a = 0; a < 4; ++a) o[a] = creal(g[a][a]);
        for (int t = 0; t < 6; ++t) {
            o[4 + 2 * t] = creal(g[pa[t]][pb[t]]);
            o[5 + 2 * t] = cimag(g[pa[t]][pb[t]]);
        }
    }
}

/* Observable identifiers (the order of the C ABI's observable bits). */
enum {
    ORC_N = 0,   /* eq. NuclearSANS                                      */
    ORC_M,       /* eq. MagneticSANS                                     */
    ORC_NM,      /* eq. NMdef (nuclear-magnetic interference)            */
    ORC_P,       /* eq. PSANSdef                                         */
    ORC_CHI,     /* eq. ChiralSANS (the real dSigma_chi/dOmega)          */
    ORC_SF,      /* eq. sfdef                                            */
    ORC_PP,      /* dSigma^{++} (Sec. 2.2)                               */
    ORC_MM,      /* dSigma^{--}                                          */
    ORC_PM,      /* dSigma^{+-}                                          */
    ORC_MP,      /* dSigma^{-+}                                          */
    ORC_PLUS,    /* SANSPOL dSigma^{+} (Sec. 2.3)                        */
    ORC_MINUS,   /* SANSPOL dSigma^{-}                                   */
    ORC_UNPOL,   /* unpolarized dSigma (Sec. 2.4)                         */
    ORC_N_OBS
};

static void cross3(const cplx a[3], const cplx b[3], cplx out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/*
 * All cross sections of Sec. 2 at one pixel from one amplitude set
 * A = (S_N, S_Mx, S_My, S_Mz) (raw sums), written as the definitions:
 *   Q = qhat x (qhat x M)                                   (eq. HJdef)
 *   N = c |S_N|^2,  M = c bH^2 |Q|^2                        (eqs. NuclearSANS, MagneticSANS)
 *   P = c bH^2 |Phat.Q|^2                                   (eq. PSANSdef)
 *   NM = c bH Phat.(S_N Q* + S_N* Q)                        (eq. NMdef)
 *   chi-term = -i c bH^2 Phat.(Q x Q*)                      (eq. ChiralSANS)
 *   sf = M - P                                              (eq. sfdef)
 *   ++ = N + NM + P, -- = N - NM + P, +- = sf + chi, -+ = sf - chi   (Sec. 2.2)
 *   + = ++ + +-, - = -- + -+                                 (Sec. 2.3)
 *   unpolarized = (++ + -- + +- + -+)/2                      (Sec. 2.4)
 * with c = scale / V.
 */
static void observables_at(const cplx A[4], const double qhat[3], double V, double bH,
                           double scale, const double Phat[3], double obs[ORC_N_OBS],
                           double *imag_residue)
{
    const double c = scale / V;
    cplx M[3] = {A[1], A[2], A[3]};
    cplx qh[3] = {qhat[0], qhat[1], qhat[2]};
    cplx t[3], Q[3];
    cross3(qh, M, t);
    cross3(qh, t, Q);

    double absQ2 = 0.0;
    for (int a = 0; a < 3; ++a) absQ2 += creal(Q[a] * conj(Q[a]));
    cplx PQ = Phat[0] * Q[0] + Phat[1] * Q[1] + Phat[2] * Q[2];
    cplx Qc[3] = {conj(Q[0]), conj(Q[1]), conj(Q[2])};
    cplx QxQc[3];
    cross3(Q, Qc, QxQc);
    cplx chi = Phat[0] * QxQc[0] + Phat[1] * QxQc[1] + Phat[2] * QxQc[2];
    cplx nm = A[0] * conj(PQ) + conj(A[0]) * PQ;
    cplx chi_term = -I * c * bH * bH * chi;

    double N = c * creal(A[0] * conj(A[0]));
    double Mg = c * bH * bH * absQ2;
    double P = c * bH * bH * creal(PQ * conj(PQ));
    double NM = c * bH * creal(nm);
    double CHI = creal(chi_term);
    double SF = Mg - P;
    double PP = N + NM + P, MM = N - NM + P, PM = SF + CHI, MP = SF - CHI;

    obs[ORC_N] = N;
    obs[ORC_M] = Mg;
    obs[ORC_NM] = NM;
    obs[ORC_P] = P;
    obs[ORC_CHI] = CHI;
    obs[ORC_SF] = SF;
    obs[ORC_PP] = PP;
    obs[ORC_MM] = MM;
    obs[ORC_PM] = PM;
    obs[ORC_MP] = MP;
    obs[ORC_PLUS] = PP + PM;
    obs[ORC_MINUS] = MM + MP;
    obs[ORC_UNPOL] = 0.5 * (PP + MM + PM + MP);
    if (imag_residue != NULL) {
        double r1 = fabs(cimag(chi_term));
        double r2 = fabs(c * bH * cimag(nm));
        *imag_residue = r1 > r2 ? r1 : r2;
    }
}

/*
 * Cross sections for n_sets amplitude sets, summed over the sets (a dilute
 * sample is sum_k obs(F_k), Sec. 3.3 dilute approximation; a single coherent
 * amplitude is n_sets = 1).  qhat is [n_pix][3].  out is [ORC_N_OBS][n_pix].
 * max_imag receives the largest imaginary residue of the terms that the
 * definitions make real (NM and the chiral term), a self-check.
 */
void orc_cross_sections(int64_t n_sets, int64_t n_pix, const double *amp_ri, const double *qhat,
                        double V, double bH, double scale, const double *Phat, double *out,
                        double *max_imag)
{
    const cplx *A = (const cplx *)amp_ri;
    double worst = 0.0;
#pragma omp parallel for reduction(max : worst)
    for (int64_t p = 0; p < n_pix; ++p) {
        double acc[ORC_N_OBS];
        for (int o = 0; o < ORC_N_OBS; ++o) acc[o] = 0.0;
        for (int64_t s = 0; s < n_sets; ++s) {
            double obs[ORC_N_OBS], res = 0.0;
            observables_at(A + (s * n_pix + p) * 4, qhat + 3 * p, V, bH, scale, Phat, obs, &res);
            for (int o = 0; o < ORC_N_OBS; ++o) acc[o] += obs[o];
            if (res > worst) worst = res;
        }
        for (int o = 0; o < ORC_N_OBS; ++o) out[o * n_pix + p] = acc[o];
    }
    if (max_imag != NULL) *max_imag = worst;
}

/*
 * Azimuthal average, eq. iqazi, I(q) = (1/2pi) int f(q, theta) dtheta.
 * Cartesian detector (kind 0): the pixels with |q| <= qmax_avg are binned in
 * n_bins equal-width annuli of [0, qmax_avg]; bin b = floor(|q| / dq) with
 * dq = qmax_avg / n_bins, |q| == qmax_avg goes to the last bin; the value is
 * the arithmetic mean of the bin (NaN and count 0 if empty).  |q| is
 * computed as sqrt(qy*qy + qz*qz) with no fused operations.
 * Polar detector (kind 1, rows = q, columns = theta on a periodic grid
 * theta_m = 2 pi m / n_theta): the trapezoidal rule over one period, which
 * on a periodic grid is the mean over theta; n_bins = rows.
 * f is [n_f][n_pix]; I is [n_f][n_bins]; count is [n_bins].
 */
void orc_azimuthal_average(int kind, int64_t n0, int64_t n1, const double *qy, const double *qz,
                           int64_t n_f, const double *f, int64_t n_bins, double qmax_avg,
                           double *Iout, int64_t *count)
{
    int64_t n_pix = n0 * n1;
    if (kind == 1) {
        for (int64_t b = 0; b < n_bins; ++b) count[b] = (b < n0) ? n1 : 0;
        for (int64_t s = 0; s < n_f; ++s)
            for (int64_t b = 0; b < n_bins; ++b) {
                if (b >= n0) { Iout[s * n_bins + b] = NAN; continue; }
                /* trapezoid over theta_0 .. theta_{n1} with f(theta_{n1}) = f(theta_0) */
                double h = 2.0 * M_PI / (double)n1, integral = 0.0;
                for (int64_t m = 0; m < n1; ++m) {
                    double f0 = f[s * n_pix + b * n1 + m];
                    double f1 = f[s * n_pix + b * n1 + ((m + 1) % n1)];
                    integral += 0.5 * h * (f0 + f1);
                }
                Iout[s * n_bins + b] = integral / (2.0 * M_PI);
            }
        return;
    }
    double dq = qmax_avg / (double)n_bins;
    int64_t *bin = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_pix > 0 ? n_pix : 1));
    for (int64_t b = 0; b < n_bins; ++b) count[b] = 0;
    for (int64_t p = 0; p < n_pix; ++p) {
        double a2 = qy[p] * qy[p];
        double b2 = qz[p] * qz[p];
        double qn = sqrt(a2 + b2); /* built with -ffp-contract=off */
        if (qn > qmax_avg) { bin[p] = -1; continue; }
        int64_t b = (int64_t)floor(qn / dq);
        if (b >= n_bins) b = n_bins - 1;
        bin[p] = b;
        count[b] += 1;
    }
    for (int64_t s = 0; s < n_f; ++s) {
        for (int64_t b = 0; b < n_bins; ++b) Iout[s * n_bins + b] = 0.0;
        for (int64_t p = 0; p < n_pix; ++p)
            if (bin[p] >= 0) Iout[s * n_bins + bin[p]] += f[s * n_pix + p];
        for (int64_t b = 0; b < n_bins; ++b)
            Iout[s * n_bins + b] = count[b] > 0 ? Iout[s * n_bins + b] / (double)count[b] : NAN;
    }
    free(bin);
}

/*
 * Correlation and pair-distance distribution functions, eqs. crrad and
 * prrad: c(r) = (scale / 2pi^2) int_0^inf I(q) j0(q r) q^2 dq, p(r) = r^2 c(r),
 * by the trapezoidal rule (Sec. 2.5) over the nodes (0, 0) and
 * (q_b, I_b q_b^2 j0(q_b r)) in the order given; samples whose I is NaN are
 * skipped.  j0(x) = sin(x)/x with j0(0) = 1.
 */
void orc_correlation(int64_t n_q, const double *q, int64_t n_f, const double *Iq, int64_t n_r,
                     const double *r, double scale, double *c, double *p)
{
    for (int64_t s = 0; s < n_f; ++s)
        for (int64_t t = 0; t < n_r; ++t) {
            double prev_q = 0.0, prev_y = 0.0, sum = 0.0;
            for (int64_t b = 0; b < n_q; ++b) {
                double Ib = Iq[s * n_q + b];
                if (isnan(Ib)) continue;
                double x = q[b] * r[t];
                double j0 = (x == 0.0) ? 1.0 : sin(x) / x;
                double y = Ib * q[b] * q[b] * j0;
                sum += 0.5 * (q[b] - prev_q) * (y + prev_y);
                prev_q = q[b];
                prev_y = y;
            }
            c[s * n_r + t] = scale * sum / (2.0 * M_PI * M_PI);
            p[s * n_r + t] = r[t] * r[t] * c[s * n_r + t];
        }
}

/*
 * Loss on the unpolarized cross section (Sec. 2.4) and its exact gradient,
 * obtained by the chain rule on the definitions (pinned in the tests by
 * finite differences):
 *   I_p = (scale/V) (|S_N|^2 + bH^2 |Q|^2),   L = sum_p w_p (I_p - T_p)^2.
 * With e_jp = exp(-i q_p . X_j) the sums are linear in the weights, so
 *   dL/dn_j   = sum_p 2 w_p (I_p - T_p) (scale/V) 2 Re(conj(S_N) e_jp),
 *   dL/dm'_ja = sum_p 2 w_p (I_p - T_p) (scale/V) bH^2 2 Re(conj(Q) . dQ/dm'_ja),
 * where dQ/dm'_ja = qhat x (qhat x (unit_a e_jp)) and m' = R m is the rotated
 * moment; the gradient with respect to the input moment is R^T dL/dm'.
 * One coherent sample (object offsets are added to the positions).
 */
void orc_loss_grad(int64_t W, const double *pos, const double *nuc, const double *mag,
                   int64_t K, const int64_t *off, const double *obj_pos, const double *R,
                   int64_t n_pix, const double *qy, const double *qz, const double *qhat,
                   double V, double bH, double scale, const double *target, const double *weight,
                   double *loss, double *dnuc, double *dmag)
{
    const double c = scale / V;
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)(n_pix * 4 + 1));
    orc_amplitudes(W, pos, nuc, mag, K, off, obj_pos, R, n_pix, qy, qz, 0, (double *)A);

    /* g_p = 2 w_p (I_p - T_p) and the magnetic interaction vector per pixel */
    double *g = (double *)malloc(sizeof(double) * (size_t)(n_pix + 1));
    cplx *Qp = (cplx *)malloc(sizeof(cplx) * (size_t)(n_pix * 3 + 1));
    double L = 0.0;
    for (int64_t p = 0; p < n_pix; ++p) {
        cplx M[3] = {A[4 * p + 1], A[4 * p + 2], A[4 * p + 3]};
        cplx qh[3] = {qhat[3 * p + 0], qhat[3 * p + 1], qhat[3 * p + 2]};
        cplx t[3], Q[3];
        cross3(qh, M, t);
        cross3(qh, t, Q);
        double absQ2 = 0.0;
        for (int a = 0; a < 3; ++a) absQ2 += creal(Q[a] * conj(Q[a]));
        double Ip = c * (creal(A[4 * p] * conj(A[4 * p])) + bH * bH * absQ2);
        double res = Ip - target[p];
        L += weight[p] * res * res;
        g[p] = 2.0 * weight[p] * res;
        for (int a = 0; a < 3; ++a) Qp[3 * p + a] = Q[a];
    }
    *loss = L;
    int64_t *kidx = object_index(W, K, off);

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < W; ++j) {
        int64_t k = kidx[j];
        double x[3] = {pos[3 * j + 0], pos[3 * j + 1], pos[3 * j + 2]};
        if (obj_pos != NULL) {
            x[0] += obj_pos[3 * k + 0];
            x[1] += obj_pos[3 * k + 1];
            x[2] += obj_pos[3 * k + 2];
        }
        double X[3];
        mat_vec(R, x, X);
        double dn = 0.0, dm_lab[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < n_pix; ++p) {
            double psi = qy[p] * X[1] + qz[p] * X[2];
            cplx e = cos(psi) - I * sin(psi);
            dn += g[p] * c * 2.0 * creal(conj(A[4 * p]) * e);
            /* |Q|^2 with Q linear in M: d|Q|^2/dm'_a = 2 Re(sum_b conj(Q_b) dQ_b/dm'_a),
               dQ/dm'_a = qhat x (qhat x (e_a e)) */
            cplx qh[3] = {qhat[3 * p + 0], qhat[3 * p + 1], qhat[3 * p + 2]};
            for (int a = 0; a < 3; ++a) {
                cplx ea[3] = {0.0, 0.0, 0.0};
                ea[a] = e;
                cplx t[3], dQ[3];
                cross3(qh, ea, t);
                cross3(qh, t, dQ);
                cplx s = 0.0;
                for (int b = 0; b < 3; ++b) s += conj(Qp[3 * p + b]) * dQ[b];
                dm_lab[a] += g[p] * c * bH * bH * 2.0 * creal(s);
            }
        }
        if (dnuc != NULL) dnuc[j] = dn;
        if (dmag != NULL) {
            /* m' = R m  =>  dL/dm = R^T dL/dm' */
            for (int b = 0; b < 3; ++b)
                dmag[3 * j + b] = R[0 * 3 + b] * dm_lab[0] + R[1 * 3 + b] * dm_lab[1] +
                                  R[2 * 3 + b] * dm_lab[2];
        }
    }
    free(A);
    free(g);
    free(Qp);
    free(kidx);
}

/*
 * Two-dimensional correlation function, eq. crav2d:
 *   C(r) = int int dSigma(q, theta) exp(i q rho cos(theta - alpha)) q dq dtheta,
 * with q rho cos(theta - alpha) = q . r for q = q (sin theta, cos theta) and
 * r = rho (sin alpha, cos alpha) in the detector plane.  The integral is the
 * quadrature sum_p wq[p] f[p] exp(i (qy[p] ry + qz[p] rz)); the trapezoidal
 * weights wq (which include the Jacobian q on a polar detector) are given by
 * the caller.  f is [n_f][n_pix]; out is [n_f][n_r] complex.
 */
void orc_correlation_2d(int64_t n_pix, const double *qy, const double *qz, const double *wq, int64_t n_f,
                        const double *f, int64_t n_r, const double *ry, const double *rz, double *out_ri)
{
    cplx *out = (cplx *)out_ri;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t s = 0; s < n_f; ++s)
        for (int64_t t = 0; t < n_r; ++t) {
            cplx acc = 0.0;
            for (int64_t p = 0; p < n_pix; ++p) {
                double phi = qy[p] * ry[t] + qz[p] * rz[t];
                acc += wq[p] * f[s * n_pix + p] * (cos(phi) + I * sin(phi));
            }
            out[s * n_r + t] = acc;
        }
}

/*
 * Modal (angular Fourier) intensities, eq. CosineSinceIntensities, on a polar
 * detector (rows q_i, columns theta_m = 2 pi m / n_theta) by the trapezoidal
 * rule over one period:
 *   I_k^{s,c}(q_i) = (2 - delta_k0)/(2 pi) int f(q_i, theta) {sin, cos}(k theta) dtheta.
 * Out: Is, Ic are [n_q][k_max+1].
 */
void orc_angular_spectrum(int64_t n_q, int64_t n_theta, const double *f, int64_t k_max,
                          double *Is, double *Ic)
{
    double h = 2.0 * M_PI / (double)n_theta;
    for (int64_t i = 0; i < n_q; ++i)
        for (int64_t k = 0; k <= k_max; ++k) {
            double ss = 0.0, cc = 0.0;
            for (int64_t m = 0; m < n_theta; ++m) {
                int64_t m1 = (m + 1) % n_theta;
                double t0 = h * (double)m, t1 = h * (double)(m + 1);
                double f0 = f[i * n_theta + m], f1 = f[i * n_theta + m1];
                ss += 0.5 * h * (f0 * sin(k * t0) + f1 * sin(k * t1));
                cc += 0.5 * h * (f0 * cos(k * t0) + f1 * cos(k * t1));
            }
            double pref = (k == 0 ? 1.0 : 2.0) / (2.0 * M_PI);
            Is[i * (k_max + 1) + k] = pref * ss;
            Ic[i * (k_max + 1) + k] = pref * cc;
        }
}
