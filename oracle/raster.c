/*
 * FP64 per-pixel compositing, adjoint and feature fusion for the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: called through ctypes by the oracle package; the
 * product library never links or calls it, and it includes nothing of it.
 *
 * Traversal (Algorithm 2): for every tile, for every pixel of the tile, walk
 * the tile's depth-sorted range front to back.  For Gaussian g at pixel centre
 * (x, y) = (px + 1/2, py + 1/2):
 *     dx = x - u_g, dy = y - v_g
 *     G  = exp(-1/2 (A dx^2 + 2 B dx dy + C dy^2))
 *     alpha = min(ALPHA_MAX, o_g G);  skip the blend if alpha < ALPHA_MIN
 *     T' = T (1 - alpha);  if T' < T_MIN stop (this Gaussian is excluded)
 *     w = alpha T;  C += w rgb_g;  F += w f_g;  T = T';  n_iter = position + 1
 * This is the colour equation of Section 3.1 with w_i = alpha_i T_i and
 * T_i = prod_{j<i} (1 - alpha_j), nearest Gaussian first.
 *
 * Adjoint (Appendix A.2, derivative of the loss with respect to alpha_k, plus
 * the final-transmittance term): with g_k = rgb_k . dC + f_k . dF,
 *     dL/dalpha_k = T_k g_k - (S_k + T_final dT) / (1 - alpha_k),
 *     S_k = sum_{i > k} w_i g_i,
 * then dL/dpower = alpha dL/dalpha and dL/do = G dL/dalpha where alpha is not
 * clamped, and power's partials in (u, v, A, B, C).  dL/drgb_k = w_k dC.
 *
 * Fusion (w-weighted transpose of feature rendering): fsum_g += w_g(p) t(p),
 * wsum_g += w_g(p).
 *
 * NDFD feature branch (Section 3.3, Appendix A.1-A.2; optional): along the
 * same walk, with unit features fh_i = f_i / |f_i| and fh_gt = F_gt / |F_gt|
 * (a zero vector's unit vector is taken as zero),
 *     sigma_i = 1 / (1 + exp(k (phi_i - lambda))),  phi_i = fh_i . fh_gt,
 *     L_gt = sum_i w_i sigma_i,
 *     L_cf = sum_i sigma_i w_i (W_{i-1} - F_{i-1} . fh_i),
 *            W_{i-1} = sum_{j<i} w_j,  F_{i-1} = sum_{j<i} w_j fh_j,
 * and, for the loss a L_gt + b L_cf of the pixel (a, b per pixel), the
 * derivative with respect to w_k in its forward-indexed form
 *     h_k = a sigma_k + b (sigma_k (W_{k-1} - F_{k-1} . fh_k)
 *                          + sum_{i>k} sigma_i w_i (1 - fh_i . fh_k)),
 * which joins g_k in the adjoint above.  sigma is a constant of the frozen
 * features, so gradients flow through w only.  Magnitude companions use
 * |fh_i . fh_j| <= 1, and sigma's companion is sigma + k sigma (1 - sigma)
 * sum_c |fh_i,c fh_gt,c|: the cosine is a sum whose rounding the sigmoid's
 * slope carries into sigma (first order).  The near-threshold bound (*_amb) does not cover these
 * terms: scenes checked with them have no near-threshold decision.
 *
 * Surfel primitive (prim = 1; oracle/surfel.py): the density is that of the
 * point of the surfel's plane that the pixel's ray meets, from the per-view
 * record (x_c, y_c, a0, a1, b0, b1, D, e1, e2):
 *     dx = x - x_c, dy = y - y_c,  k0 = dx b1 - dy a1,  k1 = dy a0 - dx b0,
 *     k2 = D - dy e1 - dx e2,  (u, v) = (k0, k1) / k2,
 *     G = exp(-(u^2 + v^2) / 2)  (0 where k2 = 0),
 * and the per-Gaussian adjoint rows hold the nine record entries, then o,
 * r, g, b (13 entries instead of 9).  Their magnitude companions carry the
 * rounding of the intersection: k0, k1, k2 by the sums of their terms'
 * magnitudes, and every division by k2 by a factor companion(k2) / k2^2.  With power = -(u^2 + v^2) / 2 and
 * lam = dL/dpower (-u / k2, -v / k2, (u^2 + v^2) / k2) = dL/dk:
 *     dL/dx_c = -(lam0 b1 - lam1 b0 - lam2 e2), dL/dy_c = -(lam1 a0 - lam0 a1 - lam2 e1),
 *     dL/da0 = lam1 dy, dL/da1 = -lam0 dy, dL/db0 = -lam1 dx, dL/db1 = lam0 dx,
 *     dL/dD = lam2, dL/de1 = -lam2 dy, dL/de2 = -lam2 dx.
 *
 * Density rounding (surfels): an FP32 implementation rounds each record entry
 * once, and near a grazing ray k2's cancellation amplifies that without bound.
 * To first order the density's relative error is den_round * gr with
 *     gr = (u^2 + v^2) / 2 + |u| um + |v| vm
 * (um, vm the companions of u, v above; den_round = a stated multiple of the
 * FP32 unit roundoff, oracle/consts.py).  An unclamped alpha inherits gr, the
 * transmittance in front of a blend tr = sum over the earlier blends of
 * alpha gr / (1 - alpha) (first order of the product of the 1 - alpha), a
 * blend weight w = alpha T the sum gr + tr.  The resulting first-order changes
 * of everything built from alpha, T and w are an absolute allowance, like the
 * near-threshold one: den_round times these sensitivities go to out_Cden,
 * out_Fden, out_Tden (forward) and are added into g2d_amb, fsum_amb and
 * wsum_amb (adjoint: the dL/dalpha, power, opacity and colour terms and the
 * fusion sums); with the NDFD branch, L_gt and L_cf get theirs
 * (out_Lgt_den, out_Lcf_den: through w_i, W_{i-1} and x_i) and the NDFD term
 * h_k of g_k its sensitivity through the other blends' w.  gr reaches 1e5 and more next to a grazing ray and stays near
 * (u^2 + v^2) / 2 for a surfel seen face-on.  A Gaussian's power is a short
 * quadratic form whose rounding stays within a few units of |power| and inside
 * the tolerance: gr = 0 there.
 *
 * Every floating-point operation is FP64.  Magnitude companions (sums of the
 * absolute values of the same terms) are accumulated alongside.
 *
 * Decisions within ambig_rel (relative) of a threshold may be taken the other
 * way by an FP32 implementation.  Such a pixel is flagged, and so is the
 * Gaussian that decides it (gflags bit 0).  Into g2d_amb / fsum_amb /
 * wsum_amb go the magnitudes of everything the other decision could change,
 * to first order: the terms the deciding Gaussian would add if it were blended
 * (its w = alpha T at the decision, with the pixel's whole suffix magnitude
 * for its S); for every contributor, the blends of deciders behind it in its
 * S, and a fraction q of its own terms, q = sum over deciders of
 * alpha / (1 - alpha) (skip rule: later transmittances scale by 1 - alpha) or
 * 1 (stop rule: the final transmittance may change entirely), at most 1.  An
 * alpha near the 0.99 clamp only switches that Gaussian's power/opacity terms
 * in that pixel; their unclamped magnitudes go to g2d_amb as well.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ALPHA_MAX 0.99
#define ALPHA_MIN (1.0 / 255.0)
#define T_MIN 1e-4

typedef struct {
    /* image and tiling */
    int64_t width, height, tile, tiles_x, tiles_y;
    int64_t d;                       /* feature channels (0 allowed) */
    double ambig_rel;                /* relative threshold distance called ambiguous */
    /* binning result for this view */
    const int64_t *ranges;           /* [tiles, 2] */
    const int64_t *list;             /* [M] Gaussian index per sorted instance */
    /* per-Gaussian projected quantities (FP64) */
    const double *u, *v, *A, *B, *C, *opac;
    const double *rgb;               /* [N, 3] */
    const double *rgb_mag;           /* [N, 3] or NULL: magnitude companion of rgb (the SH sum's
                                        terms in absolute value, plus 1/2); NULL: |rgb| */
    const double *feat;              /* [N, d] or NULL */
    /* per-pixel upstream adjoints (NULL: forward only) */
    const double *dC;                /* [P, 3] */
    const double *dF;                /* [P, d] or NULL */
    const double *dT;                /* [P] or NULL */
    const double *target;            /* [P, d] or NULL: fusion target */
    /* tiles to process (NULL: all) */
    const int64_t *tile_sel;
    int64_t n_tile_sel;
    /* per-pixel outputs */
    double *out_C;                   /* [P, 3] */
    double *out_Cmag;                /* [P, 3] or NULL: sum of w rgb_mag */
    double *out_F;                   /* [P, d] or NULL */
    double *out_Fmag;                /* [P, d] or NULL */
    double *out_T;                   /* [P] */
    int64_t *out_niter;              /* [P] */
    int32_t *out_flags;              /* [P] bit0: decision near a threshold, bit1: alpha near the clamp */
    /* per-Gaussian outputs, accumulated (caller zeroes) */
    double *g2d;                     /* [N, 9]: u v A B C o r g b, or NULL */
    double *g2d_mag;                 /* [N, 9] or NULL */
    double *fsum;                    /* [N, d] or NULL */
    double *fsum_mag;                /* [N, d] or NULL */
    double *wsum;                    /* [N] or NULL */
    double *dfeat;                   /* [N, d] or NULL: dL/df = sum_p w dF */
    double *g2d_amb;                 /* [N, 9] or NULL: magnitudes of the terms that a near-threshold
                                        decision could change (see below) */
    double *fsum_amb;                /* [N, d] or NULL: the same for the fusion sums */
    double *wsum_amb;                /* [N] or NULL: the same for the weight sums */
    int32_t *gflags;                 /* [N] or NULL: bit0 decides a near-threshold skip/stop decision
                                        (informational: bounded through the *_amb companions) */
    int64_t *counts;                 /* [3]: sum n_iter, contributing blends, alpha evaluations */
    /* NDFD feature branch (NULL ndfd_gt: off) */
    const double *ndfd_gt;           /* [P, d] ground-truth feature map F_gt */
    const double *feat_inv_norm;     /* [N] 1 / |f_g| (0 for a zero feature) */
    double ndfd_lambda, ndfd_k;      /* sigmoid threshold and slope */
    const double *ndfd_a;            /* [P] dL/dL_gt (NULL: 0) */
    const double *ndfd_b;            /* [P] dL/dL_cf (NULL: 0) */
    double *out_Lgt, *out_Lcf;       /* [P] */
    double *out_Lcf_mag;             /* [P] or NULL */
    double *out_Lgt_mag;             /* [P] or NULL */
    double *out_FN;                  /* [P, d] or NULL: sum_i w_i fh_i */
    double *out_WN;                  /* [P] or NULL: sum_i w_i */
    /* primitive: 0 Gaussian (u, v, A, B, C above), 1 surfel (srf below) */
    int64_t prim;
    const double *srf;               /* [N, 9] surfel records (prim 1) */
    /* density-rounding allowance (header): den_round 0 switches it off */
    double den_round;
    double *out_Cden;                /* [P, 3] or NULL */
    double *out_Fden;                /* [P, d] or NULL */
    double *out_Tden;                /* [P] or NULL */
    double *out_Lgt_den;             /* [P] or NULL: density-rounding allowance of L_gt (surfels) */
    double *out_Lcf_den;             /* [P] or NULL: of L_cf */
} oracle_args;

/* entries of a per-Gaussian adjoint row: (u v A B C | 9 surfel entries), o, r, g, b */
static int64_t gw_of(const oracle_args *a) { return a->prim ? 13 : 9; }

/* per-thread scratch of the NDFD branch */
typedef struct {
    double *sig, *sigm, *h, *hm, *cterm, *cmag;   /* [maxlen] per contributor */
    double *vec;                           /* [2 d] */
    double *hd;                            /* [maxlen] density-rounding sensitivity of h (surfels) */
} ndfd_scratch;

typedef struct {
    int64_t g, pos;
    double alpha, T, G, dx, dy;
    double su, sv, sk2;      /* surfel: plane coordinates and k2 */
    double ar, tr;           /* density-rounding sensitivities of alpha and of T at the blend (header) */
    int clamped, near_clamp;
} blend_rec;

/* a near-threshold decision: the deciding Gaussian, its list position, its
   state there, and whether it is the stop rule (else the skip rule) */
typedef struct {
    int64_t g, pos;
    double alpha, T, G, dx, dy;
    double su, sv, sk2;
    int stop;
    double gkm;      /* magnitude of its g_k in this pixel (filled by the adjoint) */
} amb_rec;

/* companions of a surfel's intersection at pixel offsets (dx, dy): k0, k1, k2
   are sums (companion: the sum of their terms' magnitudes) and every division
   by k2 carries k2's relative rounding, rr = companion(k2) / |k2| (first order
   of a quotient x / y: xm ym / y^2); um, vm are the companions of u, v */
static void surfel_comp(const double *r, double dx, double dy, double sk2, double *um, double *vm, double *rr) {
    const double k0m = fabs(dx * r[5]) + fabs(dy * r[3]), k1m = fabs(dy * r[2]) + fabs(dx * r[4]);
    const double k2a = fabs(sk2);
    *rr = (fabs(r[6]) + fabs(dy * r[7]) + fabs(dx * r[8])) / k2a;
    *um = k0m * *rr / k2a;
    *vm = k1m * *rr / k2a;
}

/* density of primitive g at pixel centre (x, y); the pixel offsets and (for
   surfels) the plane coordinates go to *dx, *dy, *su, *sv, *sk2, and the
   density's rounding sensitivity to *gr (0 for a Gaussian: see the header) */
static double density(const oracle_args *a, int64_t g, double x, double y, double *dx, double *dy, double *su,
                      double *sv, double *sk2, double *gr) {
    *gr = 0.0;
    if (!a->prim) {
        *dx = x - a->u[g];
        *dy = y - a->v[g];
        *su = *sv = *sk2 = 0.0;
        const double power =
            -0.5 * (a->A[g] * *dx * *dx + 2.0 * a->B[g] * *dx * *dy + a->C[g] * *dy * *dy);
        return exp(power);
    }
    const double *r = a->srf + 9 * g;
    *dx = x - r[0];
    *dy = y - r[1];
    const double k0 = *dx * r[5] - *dy * r[3];
    const double k1 = *dy * r[2] - *dx * r[4];
    const double k2 = r[6] - *dy * r[7] - *dx * r[8];
    *sk2 = k2;
    if (k2 == 0.0) {
        *su = *sv = 0.0;
        return 0.0;
    }
    *su = k0 / k2;
    *sv = k1 / k2;
    double um, vm, rr;
    surfel_comp(r, *dx, *dy, k2, &um, &vm, &rr);
    *gr = 0.5 * (*su * *su + *sv * *sv) + fabs(*su) * um + fabs(*sv) * vm;
    return exp(-0.5 * (*su * *su + *sv * *sv));
}

/* geometry entries of g's adjoint row for dL/dpower = dp at a blend (pixel
   offsets dx, dy, plane state su, sv, sk2): values into out (when dp_is_mag is
   0); else, for |dL/dpower| <= dp, the magnitudes of the terms (2: the sum of
   the absolute values of each entry's parts, what a change of dp can move)
   or their rounding companions (1: for a surfel the intersection's rounding
   carried through its quotients; for a Gaussian the same as 2); 5 entries
   for a Gaussian, 9 for a surfel */
static void geom_terms(const oracle_args *a, int64_t g, double dx, double dy, double su, double sv, double sk2,
                       double dp, int dp_is_mag, double *out) {
    if (!a->prim) {
        const double A = a->A[g], B = a->B[g], Cc = a->C[g];
        if (!dp_is_mag) {
            out[0] = dp * (A * dx + B * dy);
            out[1] = dp * (B * dx + Cc * dy);
            out[2] = dp * (-0.5 * dx * dx);
            out[3] = dp * (-dx * dy);
            out[4] = dp * (-0.5 * dy * dy);
        } else {
            out[0] = dp * (fabs(A * dx) + fabs(B * dy));
            out[1] = dp * (fabs(B * dx) + fabs(Cc * dy));
            out[2] = dp * 0.5 * dx * dx;
            out[3] = dp * fabs(dx * dy);
            out[4] = dp * 0.5 * dy * dy;
        }
        return;
    }
    const double *r = a->srf + 9 * g;
    const double a0 = r[2], a1 = r[3], b0 = r[4], b1 = r[5], e1 = r[7], e2 = r[8];
    if (sk2 == 0.0) {
        for (int k = 0; k < 9; ++k) out[k] = 0.0;
        return;
    }
    const double l0 = -su / sk2, l1 = -sv / sk2, l2 = (su * su + sv * sv) / sk2;
    if (dp_is_mag == 2) {
        const double l0a = fabs(l0), l1a = fabs(l1), l2a = fabs(l2);
        out[0] = dp * (l0a * fabs(b1) + l1a * fabs(b0) + l2a * fabs(e2));
        out[1] = dp * (l1a * fabs(a0) + l0a * fabs(a1) + l2a * fabs(e1));
        out[2] = dp * l1a * fabs(dy);
        out[3] = dp * l0a * fabs(dy);
        out[4] = dp * l1a * fabs(dx);
        out[5] = dp * l0a * fabs(dx);
        out[6] = dp * l2a;
        out[7] = dp * l2a * fabs(dy);
        out[8] = dp * l2a * fabs(dx);
    } else if (!dp_is_mag) {
        out[0] = -dp * (l0 * b1 - l1 * b0 - l2 * e2);
        out[1] = -dp * (l1 * a0 - l0 * a1 - l2 * e1);
        out[2] = dp * l1 * dy;
        out[3] = -dp * l0 * dy;
        out[4] = -dp * l1 * dx;
        out[5] = dp * l0 * dx;
        out[6] = dp * l2;
        out[7] = -dp * l2 * dy;
        out[8] = -dp * l2 * dx;
    } else {
        /* the intersection's companions; the lam's divisions by k2 carry
           k2's relative rounding rr once more */
        double um, vm, rr;
        surfel_comp(r, dx, dy, sk2, &um, &vm, &rr);
        const double k2a = fabs(sk2);
        const double l0m = um * rr / k2a, l1m = vm * rr / k2a, l2m = (um * um + vm * vm) * rr / k2a;
        (void)l0; (void)l1; (void)l2;
        out[0] = dp * (l0m * fabs(b1) + l1m * fabs(b0) + l2m * fabs(e2));
        out[1] = dp * (l1m * fabs(a0) + l0m * fabs(a1) + l2m * fabs(e1));
        out[2] = dp * l1m * fabs(dy);
        out[3] = dp * l0m * fabs(dy);
        out[4] = dp * l1m * fabs(dx);
        out[5] = dp * l0m * fabs(dx);
        out[6] = dp * l2m;
        out[7] = dp * l2m * fabs(dy);
        out[8] = dp * l2m * fabs(dx);
    }
}

static void atomic_add(double *p, double x) {
#pragma omp atomic
    *p += x;
}

static int near_rel(double x, double thr, double rel) { return fabs(x - thr) <= rel * thr; }

/* magnitude companion of rgb_g[c]: rgb is itself a sum (of SH terms) */
static double rgbm(const oracle_args *a, int64_t g, int c) {
    return a->rgb_mag ? a->rgb_mag[3 * g + c] : fabs(a->rgb[3 * g + c]);
}

/* unit feature component fh_g[c] */
static double fhat(const oracle_args *a, int64_t g, int64_t c) { return a->feat[g * a->d + c] * a->feat_inv_norm[g]; }

/* NDFD of one pixel over its contributing blends recs[0..nrec): the losses
   (and F_N, W_N), and when a or b is given, h_k for every blend. */
static void ndfd_pixel(const oracle_args *a, int64_t pix, const blend_rec *recs, int64_t nrec, ndfd_scratch *sc) {
    const int64_t d = a->d;
    const double *gt = a->ndfd_gt + pix * d;
    double gn = 0.0;
    for (int64_t c = 0; c < d; ++c) gn += gt[c] * gt[c];
    gn = sqrt(gn);
    const double ig = gn > 0.0 ? 1.0 / gn : 0.0;
    double *P = sc->vec, *B = sc->vec + d;
    memset(P, 0, sizeof(double) * d);
    double W = 0.0, Lgt = 0.0, Lgtm = 0.0, Lcf = 0.0, Lcfm = 0.0;
    /* density rounding (surfels, header): w_i moves by wd_i = w_i (ar_i + tr_i)
       to first order, W_{i-1} by Wd = the sum of the earlier wd */
    double Wd = 0.0, Lgtd = 0.0, Lcfd = 0.0;
    for (int64_t i = 0; i < nrec; ++i) {
        const int64_t g = recs[i].g;
        const double w = recs[i].alpha * recs[i].T;
        const double wd = w * (recs[i].ar + recs[i].tr);
        double phi = 0.0, phim = 0.0, pf = 0.0;
        for (int64_t c = 0; c < d; ++c) {
            phi += fhat(a, g, c) * gt[c];
            phim += fabs(fhat(a, g, c) * gt[c]);
            pf += P[c] * fhat(a, g, c);
        }
        phi *= ig;
        phim *= ig;
        const double sg = 1.0 / (1.0 + exp(a->ndfd_k * (phi - a->ndfd_lambda)));
        /* sigma's companion: sigma itself plus the cosine's companion carried
           through the sigmoid's slope k sigma (1 - sigma) */
        const double sgm = sg + a->ndfd_k * sg * (1.0 - sg) * phim;
        sc->sig[i] = sg;
        sc->sigm[i] = sgm;
        sc->cterm[i] = sg * (W - pf);
        sc->cmag[i] = sgm * 2.0 * W;
        Lgt += w * sg;
        Lgtm += w * sgm;
        Lcf += sg * w * (W - pf);
        Lcfm += sgm * w * 2.0 * W;
        Lgtd += wd * sgm;
        Lcfd += sgm * 2.0 * (wd * W + w * Wd);
        for (int64_t c = 0; c < d; ++c) P[c] += w * fhat(a, g, c);
        W += w;
        Wd += wd;
    }
    if (a->out_Lgt_den) a->out_Lgt_den[pix] = a->den_round * Lgtd;
    if (a->out_Lcf_den) a->out_Lcf_den[pix] = a->den_round * Lcfd;
    a->out_Lgt[pix] = Lgt;
    a->out_Lcf[pix] = Lcf;
    if (a->out_Lcf_mag) a->out_Lcf_mag[pix] = Lcfm;
    if (a->out_Lgt_mag) a->out_Lgt_mag[pix] = Lgtm;
    if (a->out_FN) memcpy(a->out_FN + pix * d, P, sizeof(double) * d);
    if (a->out_WN) a->out_WN[pix] = W;
    if (!a->ndfd_a && !a->ndfd_b) return;
    const double ca = a->ndfd_a ? a->ndfd_a[pix] : 0.0, cb = a->ndfd_b ? a->ndfd_b[pix] : 0.0;
    /* sum_{i>k} sigma_i w_i and sum_{i>k} sigma_i w_i fh_i, back to front; hd_k
       is h_k's density-rounding sensitivity through the other blends' w
       (W_{k-1} - x_k and A_k - y_k: 2 Wd_{k-1} and 2 sum_{i>k} sigma_i wd_i) */
    double A = 0.0, Am = 0.0, Ad = 0.0;
    memset(B, 0, sizeof(double) * d);
    for (int64_t k = nrec - 1; k >= 0; --k) {
        const int64_t g = recs[k].g;
        const double w = recs[k].alpha * recs[k].T;
        const double wd = w * (recs[k].ar + recs[k].tr);
        Wd -= wd;   /* now the sum of wd over the blends in front of k */
        double bf = 0.0;
        for (int64_t c = 0; c < d; ++c) bf += B[c] * fhat(a, g, c);
        sc->h[k] = ca * sc->sig[k] + cb * (sc->cterm[k] + (A - bf));
        sc->hm[k] = fabs(ca) * sc->sigm[k] + fabs(cb) * (sc->cmag[k] + 2.0 * Am);
        sc->hd[k] = fabs(cb) * 2.0 * (sc->sigm[k] * Wd + Ad);
        A += sc->sig[k] * w;
        Am += sc->sigm[k] * w;
        Ad += sc->sigm[k] * wd;
        for (int64_t c = 0; c < d; ++c) B[c] += sc->sig[k] * w * fhat(a, g, c);
    }
}

static void do_tile(const oracle_args *a, int64_t tile, blend_rec *recs, amb_rec *amb, double *gvec,
                    double *gmag, ndfd_scratch *sc) {
    const int64_t ty = tile / a->tiles_x, tx = tile % a->tiles_x;
    const int64_t start = a->ranges[2 * tile], end = a->ranges[2 * tile + 1];
    const int64_t d = a->d;
    int64_t local_counts[3] = {0, 0, 0};
    for (int64_t py = ty * a->tile; py < (ty + 1) * a->tile && py < a->height; ++py) {
        for (int64_t px = tx * a->tile; px < (tx + 1) * a->tile && px < a->width; ++px) {
            const int64_t pix = py * a->width + px;
            const double x = (double)px + 0.5, y = (double)py + 0.5;
            double T = 1.0, col[3] = {0, 0, 0}, colm[3] = {0, 0, 0};
            double *F = a->out_F ? a->out_F + pix * d : NULL;
            double *Fm = a->out_Fmag ? a->out_Fmag + pix * d : NULL;
            if (F) memset(F, 0, sizeof(double) * d);
            if (Fm) memset(Fm, 0, sizeof(double) * d);
            int64_t niter = 0, nrec = 0, namb = 0;
            int32_t flags = 0;
            double tau = 0.0;   /* density-rounding sensitivity of T (header) */
            double cden[3] = {0, 0, 0};
            double *Fd = a->out_Fden ? a->out_Fden + pix * d : NULL;
            if (Fd) memset(Fd, 0, sizeof(double) * d);
            /* ---- forward, front to back ---- */
            for (int64_t pos = start; pos < end; ++pos) {
                const int64_t g = a->list[pos];
                double dx, dy, su, sv, sk2, gr;
                const double G = density(a, g, x, y, &dx, &dy, &su, &sv, &sk2, &gr);
                const double raw = a->opac[g] * G;
                const double alpha = raw < ALPHA_MAX ? raw : ALPHA_MAX;
                const double ar = raw < ALPHA_MAX ? gr : 0.0;
                local_counts[2]++;
                /* a decision this close to its threshold may go either way in FP32:
                   the clamp only changes g's own terms in this pixel (pixel bit 1,
                   bounded through g2d_amb); the skip and stop rules change the
                   whole pixel (pixel bit 0) */
                if (near_rel(raw, ALPHA_MAX, a->ambig_rel)) flags |= 2;
                if (near_rel(alpha, ALPHA_MIN, a->ambig_rel)) {
                    flags |= 1;
                    amb[namb++] = (amb_rec){g, pos, alpha, T, G, dx, dy, su, sv, sk2, 0, 0.0};
                }
                if (alpha < ALPHA_MIN) continue;
                const double Tn = T * (1.0 - alpha);
                if (near_rel(Tn, T_MIN, a->ambig_rel)) {
                    flags |= 1;
                    amb[namb++] = (amb_rec){g, pos, alpha, T, G, dx, dy, su, sv, sk2, 1, 0.0};
                }
                if (Tn < T_MIN) break;
                const double w = alpha * T, wd = w * (ar + tau);
                for (int c = 0; c < 3; ++c) {
                    col[c] += w * a->rgb[3 * g + c];
                    colm[c] += w * rgbm(a, g, c);
                    cden[c] += wd * rgbm(a, g, c);
                }
                if (F && a->feat)
                    for (int64_t k = 0; k < d; ++k) F[k] += w * a->feat[g * d + k];
                if (Fm && a->feat)
                    for (int64_t k = 0; k < d; ++k) Fm[k] += w * fabs(a->feat[g * d + k]);
                if (Fd && a->feat)
                    for (int64_t k = 0; k < d; ++k) Fd[k] += wd * fabs(a->feat[g * d + k]) * a->den_round;
                blend_rec *r = &recs[nrec++];
                r->g = g; r->pos = pos; r->alpha = alpha; r->T = T; r->G = G; r->dx = dx; r->dy = dy;
                r->su = su; r->sv = sv; r->sk2 = sk2; r->ar = ar; r->tr = tau;
                tau += alpha * ar / (1.0 - alpha);
                r->clamped = raw >= ALPHA_MAX;
                r->near_clamp = near_rel(raw, ALPHA_MAX, a->ambig_rel);
                T = Tn;
                niter = pos - start + 1;
                local_counts[1]++;
            }
            local_counts[0] += niter;
            for (int c = 0; c < 3; ++c) a->out_C[3 * pix + c] = col[c];
            if (a->out_Cmag)
                for (int c = 0; c < 3; ++c) a->out_Cmag[3 * pix + c] = colm[c];
            a->out_T[pix] = T;
            if (a->out_Tden) a->out_Tden[pix] = a->den_round * T * tau;
            if (a->out_Cden)
                for (int c = 0; c < 3; ++c) a->out_Cden[3 * pix + c] = a->den_round * cden[c];
            a->out_niter[pix] = niter;
            if (a->out_flags) a->out_flags[pix] = flags;
            /* the Gaussians that decide a near-threshold skip/stop may gain or lose
               this pixel's whole contribution: flag them; the other contributors of
               such a pixel are bounded through the *_amb companions below */
            if ((flags & 1) && a->gflags) {
                for (int64_t i = 0; i < namb; ++i) {
#pragma omp atomic
                    a->gflags[amb[i].g] |= 1;
                }
            }
            const int ndfd_grad = a->ndfd_gt && (a->ndfd_a || a->ndfd_b);
            if (a->ndfd_gt) ndfd_pixel(a, pix, recs, nrec, sc);
            if (!a->dC) continue;
            /* ---- adjoint, back to front over the contributing blends ---- */
            const double *dC = a->dC + 3 * pix;
            const double *dF = (a->dF && a->feat) ? a->dF + pix * d : NULL;
            const double dT = a->dT ? a->dT[pix] : 0.0;
            const double *tgt = a->target ? a->target + pix * d : NULL;
            const double Tfin = T;
            double S = 0.0, Sm = 0.0, Sd = 0.0;
            /* another skip decision by decider j scales every later T (and T_final)
               by (1 - alpha_j), i.e. changes them by at most alpha_j / (1 - alpha_j)
               relative; another stop decision changes T_final by up to 100%; q is
               the sum over the pixel's deciders (at most 1) */
            double q = 0.0;
            if (flags & 1) {
                for (int64_t i = 0; i < namb; ++i) {
                    amb_rec *e = &amb[i];
                    q += e->stop ? 1.0 : e->alpha / (1.0 - e->alpha);
                    double gkm = 0.0;
                    for (int c = 0; c < 3; ++c) gkm += rgbm(a, e->g, c) * fabs(dC[c]);
                    if (dF)
                        for (int64_t k = 0; k < d; ++k) gkm += fabs(a->feat[e->g * d + k] * dF[k]);
                    e->gkm = gkm;
                }
                if (q > 1.0) q = 1.0;
            }
            for (int64_t i = nrec - 1; i >= 0; --i) {
                const blend_rec *r = &recs[i];
                const int64_t g = r->g;
                const double w = r->alpha * r->T;
                double gk = 0.0, gkm = 0.0;
                for (int c = 0; c < 3; ++c) {
                    gk += a->rgb[3 * g + c] * dC[c];
                    gkm += rgbm(a, g, c) * fabs(dC[c]);
                }
                if (dF)
                    for (int64_t k = 0; k < d; ++k) {
                        gk += a->feat[g * d + k] * dF[k];
                        gkm += fabs(a->feat[g * d + k] * dF[k]);
                    }
                double gkd = 0.0;   /* density-rounding sensitivity of g_k itself (NDFD terms) */
                if (ndfd_grad) {
                    gk += sc->h[i];
                    gkm += sc->hm[i];
                    gkd = sc->hd[i];
                }
                const double inv1ma = 1.0 / (1.0 - r->alpha);
                const double dalpha = r->T * gk - (S + Tfin * dT) * inv1ma;
                const double dalpham = r->T * gkm + (Sm + Tfin * fabs(dT)) * inv1ma;
                /* density-rounding sensitivity of dL/dalpha: T's, S's and Tfin's,
                   and that of 1 / (1 - alpha) */
                const double dalphad = r->T * (r->tr * gkm + gkd) + (Sd + Tfin * tau * fabs(dT)) * inv1ma +
                                       (Sm + Tfin * fabs(dT)) * inv1ma * r->alpha * r->ar * inv1ma;
                const double wd = w * (r->ar + r->tr);
                S += w * gk;
                Sm += w * gkm;
                Sd += wd * gkm + w * gkd;
                double dpow = 0.0, dpowm = 0.0, dop = 0.0, dopm = 0.0, dpowd = 0.0, dopd = 0.0;
                if (!r->clamped) {
                    dpow = dalpha * r->alpha;
                    dpowm = dalpham * r->alpha;
                    dop = dalpha * r->G;
                    dopm = dalpham * r->G;
                    dpowd = (dalphad + dalpham * r->ar) * r->alpha;
                    dopd = (dalphad + dalpham * r->ar) * r->G;
                }
                /* power's partials (Gaussian: power = -1/2 (A dx^2 + 2 B dx dy + C dy^2),
                   dx = x - u; surfel: see the header), then o and the colour */
                const int64_t gw = gw_of(a), ng = gw - 4;
                geom_terms(a, g, r->dx, r->dy, r->su, r->sv, r->sk2, dpow, 0, gvec);
                geom_terms(a, g, r->dx, r->dy, r->su, r->sv, r->sk2, dpowm, 1, gmag);
                gvec[ng] = dop;
                gmag[ng] = dopm;
                for (int c = 0; c < 3; ++c) {
                    gvec[ng + 1 + c] = w * dC[c];
                    gmag[ng + 1 + c] = fabs(w * dC[c]);
                }
                if (a->g2d)
                    for (int64_t k = 0; k < gw; ++k) atomic_add(&a->g2d[gw * g + k], gvec[k]);
                if (a->g2d_mag)
                    for (int64_t k = 0; k < gw; ++k) atomic_add(&a->g2d_mag[gw * g + k], gmag[k]);
                if (a->g2d_amb && a->den_round > 0.0 && (dalphad > 0.0 || wd > 0.0)) {
                    double am[13];
                    geom_terms(a, g, r->dx, r->dy, r->su, r->sv, r->sk2, a->den_round * dpowd, 2, am);
                    am[ng] = a->den_round * dopd;
                    for (int c = 0; c < 3; ++c) am[ng + 1 + c] = a->den_round * fabs(wd * dC[c]);
                    for (int64_t k = 0; k < gw; ++k) atomic_add(&a->g2d_amb[gw * g + k], am[k]);
                }
                /* what a decision taken the other way in FP32 can change in this
                   contributor's terms: in an ambiguous pixel, q of its dL/dalpha
                   magnitude plus the blend each decider behind it would add to its
                   S, and q of its colour terms; near the clamp, its unclamped
                   power/opacity terms */
                if (a->g2d_amb && ((flags & 1) || r->near_clamp)) {
                    double damb = 0.0;
                    if (flags & 1) {
                        double extra = 0.0;
                        for (int64_t j = 0; j < namb; ++j)
                            if (amb[j].pos > r->pos) extra += amb[j].alpha * amb[j].T * amb[j].gkm;
                        damb += q * dalpham + extra * inv1ma;
                    }
                    if (r->near_clamp) damb += dalpham;
                    const double um = damb * r->alpha, om = damb * r->G;
                    double am[13];
                    geom_terms(a, g, r->dx, r->dy, r->su, r->sv, r->sk2, um, 2, am);
                    am[ng] = om;
                    for (int c = 0; c < 3; ++c) am[ng + 1 + c] = (flags & 1) ? q * gmag[ng + 1 + c] : 0.0;
                    for (int64_t k = 0; k < gw; ++k) atomic_add(&a->g2d_amb[gw * g + k], am[k]);
                }
                if (a->dfeat && dF)
                    for (int64_t k = 0; k < d; ++k) atomic_add(&a->dfeat[g * d + k], w * dF[k]);
                if (tgt) {
                    if (a->fsum)
                        for (int64_t k = 0; k < d; ++k) atomic_add(&a->fsum[g * d + k], w * tgt[k]);
                    if (a->fsum_mag)
                        for (int64_t k = 0; k < d; ++k) atomic_add(&a->fsum_mag[g * d + k], fabs(w * tgt[k]));
                    if (a->wsum) atomic_add(&a->wsum[g], w);
                    if (wd > 0.0 && a->den_round > 0.0) {
                        if (a->fsum_amb)
                            for (int64_t k = 0; k < d; ++k)
                                atomic_add(&a->fsum_amb[g * d + k], a->den_round * fabs(wd * tgt[k]));
                        if (a->wsum_amb) atomic_add(&a->wsum_amb[g], a->den_round * wd);
                    }
                    if (flags & 1) {
                        if (a->fsum_amb)
                            for (int64_t k = 0; k < d; ++k) atomic_add(&a->fsum_amb[g * d + k], q * fabs(w * tgt[k]));
                        if (a->wsum_amb) atomic_add(&a->wsum_amb[g], q * w);
                    }
                }
            }
            /* each decider may gain (or keep) a blend here in FP32 that FP64 did
               not take: bound the terms such a blend would add, with the whole
               suffix magnitude of the pixel standing in for its S */
            for (int64_t i = 0; i < namb; ++i) {
                const amb_rec *e = &amb[i];
                const int64_t g = e->g;
                const double gkm = e->gkm;
                const double w = e->alpha * e->T;
                const double dalpham = e->T * gkm + (Sm + Tfin * fabs(dT)) / (1.0 - e->alpha);
                const double um = dalpham * e->alpha, om = dalpham * e->G;
                if (a->g2d_amb) {
                    const int64_t gw = gw_of(a), ng = gw - 4;
                    double am[13];
                    geom_terms(a, g, e->dx, e->dy, e->su, e->sv, e->sk2, um, 2, am);
                    am[ng] = om;
                    for (int c = 0; c < 3; ++c) am[ng + 1 + c] = w * fabs(dC[c]);
                    for (int64_t k = 0; k < gw; ++k) atomic_add(&a->g2d_amb[gw * g + k], am[k]);
                }
                if (tgt) {
                    if (a->fsum_amb)
                        for (int64_t k = 0; k < d; ++k) atomic_add(&a->fsum_amb[g * d + k], fabs(w * tgt[k]));
                    if (a->wsum_amb) atomic_add(&a->wsum_amb[g], w);
                }
            }
        }
    }
    if (a->counts)
        for (int k = 0; k < 3; ++k) {
#pragma omp atomic
            a->counts[k] += local_counts[k];
        }
}

int oracle_raster(const oracle_args *a) {
    const int64_t ntiles = a->tiles_x * a->tiles_y;
    const int64_t nsel = a->tile_sel ? a->n_tile_sel : ntiles;
    int64_t maxlen = 0;
    for (int64_t i = 0; i < nsel; ++i) {
        const int64_t t = a->tile_sel ? a->tile_sel[i] : i;
        const int64_t len = a->ranges[2 * t + 1] - a->ranges[2 * t];
        if (len > maxlen) maxlen = len;
    }
    int err = 0;
#pragma omp parallel
    {
        blend_rec *recs = (blend_rec *)malloc(sizeof(blend_rec) * (size_t)(maxlen + 1));
        amb_rec *amb = (amb_rec *)malloc(sizeof(amb_rec) * (size_t)(2 * maxlen + 2));
        double *nd = (double *)malloc(sizeof(double) * (size_t)(7 * (maxlen + 1) + 2 * (a->d + 1)));
        ndfd_scratch sc = {nd, nd + (maxlen + 1), nd + 2 * (maxlen + 1), nd + 3 * (maxlen + 1),
                           nd + 4 * (maxlen + 1), nd + 5 * (maxlen + 1), nd + 6 * (maxlen + 1),
                           nd + 6 * (maxlen + 1) + 2 * (a->d + 1)};
        double gvec[13], gmag[13];
        if (!recs || !amb || !nd) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < nsel; ++i)
                do_tile(a, a->tile_sel ? a->tile_sel[i] : i, recs, amb, gvec, gmag, &sc);
        }
        free(recs);
        free(amb);
        free(nd);
    }
    return err;
}

int oracle_num_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

/* Number of OpenMP threads for later calls (timing on one core or all). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
