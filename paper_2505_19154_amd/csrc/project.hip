// Projection of every (view, Gaussian) to the screen, and its adjoint.
//
// Forward (Algorithm 2, Homogenization + 2DScreenGaussians; the screen-space
// Gaussian of Section 3.1):
//   * binning quantities (depth key, tile rect) in float32 with a fixed
//     operation order and no contraction, so that the keys are reproducible
//     bit for bit;
//   * the 2D covariance Sigma2 = J W Sigma3 W^T J^T + 0.3 I, its inverse and
//     the inverse's eigenframe in FP64 (the one FP64 block of the path: the
//     covariance can be nearly singular for thin, edge-on Gaussians);
//   * the mean (u, v) from the FP64 camera-space centre, stored as a float
//     pair hi + lo so that pixel offsets keep full FP32 accuracy at 1080p;
//   * view-dependent colour from real SH of degree <= 3 in FP32.
// One thread per (view, Gaussian); SoA inputs, coalesced record writes.
#include "kernels.hpp"

namespace fh {

struct BinQ {
    float depth, u, v, ex, ey;
    int x0, y0, x1, y1;
    bool binned;
};

// Natural log of a finite float32 x > 1 by basic float32 operations only, so
// that the result is reproducible bit for bit: x = m 2^e (exact), m brought
// into [sqrt(1/2), sqrt 2) (exact halving), then ln m = 2 atanh(s),
// s = (m - 1)/(m + 1), by the series s (1 + s^2/3 + s^4/5 + s^6/7 + s^8/9)
// in Horner form (|s| <= 0.1716: the next term is below float32 resolution).
// The constants are the float32 roundings of the double values.
__device__ float ln_f32_ops(float x) {
#pragma clang fp contract(off)
    const uint32_t bits = __float_as_uint(x);
    int e = (int)(bits >> 23) - 127;
    float m = __uint_as_float((bits & 0x7FFFFFu) | 0x3F800000u);
    if (m > (float)1.4142135) {
        m = m * 0.5f;
        e += 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    const float p = ((((float)(1.0 / 9.0) * z + (float)(1.0 / 7.0)) * z + (float)(1.0 / 5.0)) * z +
                     (float)(1.0 / 3.0)) * z + 1.0f;
    return (float)e * (float)0.6931472 + (s + s) * p;
}

// The float32 binning chain.  Every line is one IEEE float32 operation in the
// written order; contraction into FMA is disabled.  Box factor: 11.1 for every
// Gaussian (FH_BIN_BOX), or min(11.1, 2 ln(255 o) + 1/256) with no instances
// where 255 o <= 1 (FH_BIN_OPACITY: alpha = o G reaches 1/255 only where
// d^T Sigma2^-1 d <= 2 ln(255 o)).
__device__ BinQ binning_f32(float mx, float my, float mz, float sx, float sy, float sz, float qw, float qx,
                            float qy, float qz, float op, int rule, const fh_camera& c, int tiles_x, int tiles_y) {
#pragma clang fp contract(off)
    const float* R = c.R;
    const float px = ((R[0] * mx + R[1] * my) + R[2] * mz) + c.t[0];
    const float py = ((R[3] * mx + R[4] * my) + R[5] * mz) + c.t[1];
    const float pz = ((R[6] * mx + R[7] * my) + R[8] * mz) + c.t[2];
    BinQ b;
    b.depth = pz;
    const bool visible = pz > Z_NEAR;
    b.u = (c.fx * px) / pz + c.cx;
    b.v = (c.fy * py) / pz + c.cy;

    const float n = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    const float k = 2.0f / n;
    float Rq[9];
    Rq[0] = 1.0f - k * (qy * qy + qz * qz);
    Rq[1] = k * (qx * qy - qw * qz);
    Rq[2] = k * (qx * qz + qw * qy);
    Rq[3] = k * (qx * qy + qw * qz);
    Rq[4] = 1.0f - k * (qx * qx + qz * qz);
    Rq[5] = k * (qy * qz - qw * qx);
    Rq[6] = k * (qx * qz - qw * qy);
    Rq[7] = k * (qy * qz + qw * qx);
    Rq[8] = 1.0f - k * (qx * qx + qy * qy);
    const float s[3] = {sx, sy, sz};
    float M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * s[j];

    const float j00 = c.fx / pz;
    const float j11 = c.fy / pz;
    const float j02 = -(j00 * px) / pz;
    const float j12 = -(j11 * py) / pz;
    float T0[3], T1[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        T0[kk] = j00 * R[kk] + j02 * R[6 + kk];
        T1[kk] = j11 * R[3 + kk] + j12 * R[6 + kk];
    }
    float W0[3], W1[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        W0[l] = (T0[0] * M[l] + T0[1] * M[3 + l]) + T0[2] * M[6 + l];
        W1[l] = (T1[0] * M[l] + T1[1] * M[3 + l]) + T1[2] * M[6 + l];
    }
    const float a = ((W0[0] * W0[0] + W0[1] * W0[1]) + W0[2] * W0[2]) + LOWPASS;
    const float cc = ((W1[0] * W1[0] + W1[1] * W1[1]) + W1[2] * W1[2]) + LOWPASS;
    float kap = KAPPA;
    bool live = true;
    if (rule == FH_BIN_OPACITY) {
        const float x = 255.0f * op;
        live = x > 1.0f;
        const float lx = ln_f32_ops(live ? x : 2.0f);
        kap = live ? fminf((lx + lx) + 0.00390625f, KAPPA) : 0.0f;
    }
    b.ex = sqrtf(kap * a);
    b.ey = sqrtf(kap * cc);

    const float ts = (float)TILE;
    const float x0f = floorf((b.u - b.ex) / ts);
    const float x1f = floorf((b.u + b.ex) / ts);
    const float y0f = floorf((b.v - b.ey) / ts);
    const float y1f = floorf((b.v + b.ey) / ts);
    const bool finite = isfinite(b.u) && isfinite(b.v) && isfinite(b.ex) && isfinite(b.ey);
    const bool ok = visible && finite && live;
    b.x0 = ok ? (int)fmaxf(x0f, 0.0f) : 0;
    b.x1 = ok ? (int)fminf(x1f, (float)(tiles_x - 1)) : -1;
    b.y0 = ok ? (int)fmaxf(y0f, 0.0f) : 0;
    b.y1 = ok ? (int)fminf(y1f, (float)(tiles_y - 1)) : -1;
    b.binned = ok && b.x0 <= b.x1 && b.y0 <= b.y1;
    return b;
}

// Surfel binning (Section 3.1's planar primitive), float32 chain, contraction
// disabled, every line one IEEE operation in the written order.  Camera-space
// scaled tangents T_u = s_u R_c t_u, T_v = s_v R_c t_v (t_u, t_v: columns 0
// and 1 of R_q); the surfel map in pixel offsets from the projected centre,
//   a_i = fx (T_i.x p_z - p_x T_i.z) / p_z^2,  b_i = fy (T_i.y p_z - p_y T_i.z) / p_z^2,
//   c_i = T_i.z / p_z,
// and the bounding box of the image of the disc u^2 + v^2 <= kappa (the
// opacity-aware kappa) from its dual conic D = kappa (a a, a.b, a.c; b b,
// b.c; c c) - e3 e3^T: dx = (D02 -+ sqrt(D02^2 - D00 D22)) / D22, dy likewise;
// the disc lies in front of the camera iff D22 < 0 (else culled).
__device__ BinQ binning_surfel_f32(float mx, float my, float mz, float sx, float sy, float qw, float qx, float qy,
                                   float qz, float op, const fh_camera& c, int tiles_x, int tiles_y) {
#pragma clang fp contract(off)
    const float* R = c.R;
    const float px = ((R[0] * mx + R[1] * my) + R[2] * mz) + c.t[0];
    const float py = ((R[3] * mx + R[4] * my) + R[5] * mz) + c.t[1];
    const float pz = ((R[6] * mx + R[7] * my) + R[8] * mz) + c.t[2];
    BinQ b;
    b.depth = pz;
    const bool visible = pz > Z_NEAR;
    b.u = (c.fx * px) / pz + c.cx;
    b.v = (c.fy * py) / pz + c.cy;
    const float n = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    const float k = 2.0f / n;
    // columns 0 and 1 of R_q
    const float r00 = 1.0f - k * (qy * qy + qz * qz), r10 = k * (qx * qy + qw * qz), r20 = k * (qx * qz - qw * qy);
    const float r01 = k * (qx * qy - qw * qz), r11 = 1.0f - k * (qx * qx + qz * qz), r21 = k * (qy * qz + qw * qx);
    float tu[3], tv[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        tu[r] = ((R[3 * r] * r00 + R[3 * r + 1] * r10) + R[3 * r + 2] * r20) * sx;
        tv[r] = ((R[3 * r] * r01 + R[3 * r + 1] * r11) + R[3 * r + 2] * r21) * sy;
    }
    const float zz = pz * pz;
    const float a0 = c.fx * ((tu[0] * pz - px * tu[2]) / zz);
    const float a1 = c.fx * ((tv[0] * pz - px * tv[2]) / zz);
    const float b0 = c.fy * ((tu[1] * pz - py * tu[2]) / zz);
    const float b1 = c.fy * ((tv[1] * pz - py * tv[2]) / zz);
    const float c0 = tu[2] / pz;
    const float c1 = tv[2] / pz;
    const float x = 255.0f * op;
    const bool live = x > 1.0f;
    const float lx = ln_f32_ops(live ? x : 2.0f);
    const float kap = live ? fminf((lx + lx) + 0.00390625f, KAPPA) : 0.0f;
    const float d00 = kap * (a0 * a0 + a1 * a1);
    const float d02 = kap * (a0 * c0 + a1 * c1);
    const float d11 = kap * (b0 * b0 + b1 * b1);
    const float d12 = kap * (b0 * c0 + b1 * c1);
    const float d22 = kap * (c0 * c0 + c1 * c1) - 1.0f;
    const bool front = d22 < 0.0f;
    const float sxr = sqrtf(d02 * d02 - d00 * d22);
    const float syr = sqrtf(d12 * d12 - d11 * d22);
    const float xlo = (d02 + sxr) / d22, xhi = (d02 - sxr) / d22;
    const float ylo = (d12 + syr) / d22, yhi = (d12 - syr) / d22;
    const float ts = (float)TILE;
    const float x0f = floorf((b.u + xlo) / ts);
    const float x1f = floorf((b.u + xhi) / ts);
    const float y0f = floorf((b.v + ylo) / ts);
    const float y1f = floorf((b.v + yhi) / ts);
    const bool finite = isfinite(b.u) && isfinite(b.v) && isfinite(xlo) && isfinite(xhi) && isfinite(ylo) &&
                        isfinite(yhi);
    const bool ok = visible && finite && live && front;
    b.ex = b.ey = 0.0f;
    b.x0 = ok ? (int)fmaxf(x0f, 0.0f) : 0;
    b.x1 = ok ? (int)fminf(x1f, (float)(tiles_x - 1)) : -1;
    b.y0 = ok ? (int)fmaxf(y0f, 0.0f) : 0;
    b.y1 = ok ? (int)fminf(y1f, (float)(tiles_y - 1)) : -1;
    b.binned = ok && b.x0 <= b.x1 && b.y0 <= b.y1;
    return b;
}

// Real spherical harmonics (orthonormal, Condon-Shortley phase, index
// l*l + m + l) as Cartesian polynomials of the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
    Y[0] = 0.28209479177387814f;
    if (deg < 1) return;
    Y[1] = -0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = -0.48860251190291992f * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = -1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * x * z;
    Y[8] = 0.54627421529603959f * (xx - yy);
    if (deg < 3) return;
    Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
    Y[10] = 2.8906114426405538f * x * y * z;
    Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.4453057213202769f * z * (xx - yy);
    Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

// Gradient of the polynomials above with respect to (x, y, z): G[b][0..2].
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float (*G)[3]) {
    G[0][0] = G[0][1] = G[0][2] = 0.0f;
    if (deg < 1) return;
    const float c1 = 0.48860251190291992f;
    G[1][0] = 0.0f; G[1][1] = -c1; G[1][2] = 0.0f;
    G[2][0] = 0.0f; G[2][1] = 0.0f; G[2][2] = c1;
    G[3][0] = -c1; G[3][1] = 0.0f; G[3][2] = 0.0f;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.54627421529603959f;
    G[4][0] = c2a * y; G[4][1] = c2a * x; G[4][2] = 0.0f;
    G[5][0] = 0.0f; G[5][1] = -c2a * z; G[5][2] = -c2a * y;
    G[6][0] = -2.0f * c2b * x; G[6][1] = -2.0f * c2b * y; G[6][2] = 4.0f * c2b * z;
    G[7][0] = -c2a * z; G[7][1] = 0.0f; G[7][2] = -c2a * x;
    G[8][0] = 2.0f * c2c * x; G[8][1] = -2.0f * c2c * y; G[8][2] = 0.0f;
    if (deg < 3) return;
    const float c3a = 0.59004358992664352f, c3b = 2.8906114426405538f, c3c = 0.45704579946446572f,
                c3d = 0.37317633259011540f, c3e = 1.4453057213202769f;
    // Y9 = -c3a (3 x^2 y - y^3)
    G[9][0] = -c3a * 6.0f * x * y; G[9][1] = -c3a * (3.0f * xx - 3.0f * yy); G[9][2] = 0.0f;
    // Y10 = c3b x y z
    G[10][0] = c3b * y * z; G[10][1] = c3b * x * z; G[10][2] = c3b * x * y;
    // Y11 = -c3c (4 y z^2 - x^2 y - y^3)
    G[11][0] = c3c * 2.0f * x * y; G[11][1] = -c3c * (4.0f * zz - xx - 3.0f * yy); G[11][2] = -c3c * 8.0f * y * z;
    // Y12 = c3d (2 z^3 - 3 x^2 z - 3 y^2 z)
    G[12][0] = -c3d * 6.0f * x * z; G[12][1] = -c3d * 6.0f * y * z; G[12][2] = c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
    // Y13 = -c3c (4 x z^2 - x^3 - x y^2)
    G[13][0] = -c3c * (4.0f * zz - 3.0f * xx - yy); G[13][1] = c3c * 2.0f * x * y; G[13][2] = -c3c * 8.0f * x * z;
    // Y14 = c3e (x^2 z - y^2 z)
    G[14][0] = c3e * 2.0f * x * z; G[14][1] = -c3e * 2.0f * y * z; G[14][2] = c3e * (xx - yy);
    // Y15 = -c3a (x^3 - 3 x y^2)
    G[15][0] = -c3a * (3.0f * xx - 3.0f * yy); G[15][1] = c3a * 6.0f * x * y; G[15][2] = 0.0f;
}

// FP64 screen-space covariance for one (camera, Gaussian): camera-space
// centre p, Sigma2 entries (a, b, c) including the low-pass, and the pieces
// the adjoint reuses.
struct Cov64 {
    double p[3];
    double T[2][3];   // J R_c
    double M[3][3];   // R_q diag(s)
    double Rq[3][3];
    double qn[4], qnorm;
    double W[2][3];   // T M
    double a, b, c;
};

__device__ Cov64 cov64(const float* mu, const float* sc, const float* q, const fh_camera& cam) {
    Cov64 o;
    const float* R = cam.R;
    for (int r = 0; r < 3; ++r)
        o.p[r] = (double)R[3 * r] * mu[0] + (double)R[3 * r + 1] * mu[1] + (double)R[3 * r + 2] * mu[2] + (double)cam.t[r];
    const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    o.qnorm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double w = qw / o.qnorm, x = qx / o.qnorm, y = qy / o.qnorm, z = qz / o.qnorm;
    o.qn[0] = w; o.qn[1] = x; o.qn[2] = y; o.qn[3] = z;
    o.Rq[0][0] = 1 - 2 * (y * y + z * z); o.Rq[0][1] = 2 * (x * y - w * z); o.Rq[0][2] = 2 * (x * z + w * y);
    o.Rq[1][0] = 2 * (x * y + w * z); o.Rq[1][1] = 1 - 2 * (x * x + z * z); o.Rq[1][2] = 2 * (y * z - w * x);
    o.Rq[2][0] = 2 * (x * z - w * y); o.Rq[2][1] = 2 * (y * z + w * x); o.Rq[2][2] = 1 - 2 * (x * x + y * y);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) o.M[i][j] = o.Rq[i][j] * (double)sc[j];
    const double fx = cam.fx, fy = cam.fy, pz = o.p[2];
    const double j00 = fx / pz, j02 = -fx * o.p[0] / (pz * pz);
    const double j11 = fy / pz, j12 = -fy * o.p[1] / (pz * pz);
    for (int k = 0; k < 3; ++k) {
        o.T[0][k] = j00 * R[k] + j02 * R[6 + k];
        o.T[1][k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    for (int r = 0; r < 2; ++r)
        for (int l = 0; l < 3; ++l) o.W[r][l] = o.T[r][0] * o.M[0][l] + o.T[r][1] * o.M[1][l] + o.T[r][2] * o.M[2][l];
    o.a = o.W[0][0] * o.W[0][0] + o.W[0][1] * o.W[0][1] + o.W[0][2] * o.W[0][2] + LOWPASS_D;
    o.b = o.W[0][0] * o.W[1][0] + o.W[0][1] * o.W[1][1] + o.W[0][2] * o.W[1][2];
    o.c = o.W[1][0] * o.W[1][0] + o.W[1][1] * o.W[1][1] + o.W[1][2] * o.W[1][2] + LOWPASS_D;
    return o;
}

__device__ __forceinline__ void cam_centre(const fh_camera& c, float* cp) {
    const float* R = c.R;
    for (int k = 0; k < 3; ++k) cp[k] = -(R[k] * c.t[0] + R[3 + k] * c.t[1] + R[6 + k] * c.t[2]);
}

// FP64 surfel frame for one (camera, surfel): camera-space centre p, the
// camera-space tangent directions du = R_c t_u, dv = R_c t_v, the scaled
// tangents T_u = s_u du, T_v = s_v dv, and the record entries a, b, c of the
// surfel map in pixel offsets from the projected centre (see binning_surfel_f32).
struct Srf64 {
    double p[3], du[3], dv[3], Tu[3], Tv[3];
    double qn[4], qnorm;
    double a0, a1, b0, b1, c0, c1;
};

__device__ Srf64 srf64(const float* mu, const float* sc, const float* q, const fh_camera& cam) {
    Srf64 o;
    const float* R = cam.R;
    for (int r = 0; r < 3; ++r)
        o.p[r] = (double)R[3 * r] * mu[0] + (double)R[3 * r + 1] * mu[1] + (double)R[3 * r + 2] * mu[2] + (double)cam.t[r];
    const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    o.qnorm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double w = qw / o.qnorm, x = qx / o.qnorm, y = qy / o.qnorm, z = qz / o.qnorm;
    o.qn[0] = w; o.qn[1] = x; o.qn[2] = y; o.qn[3] = z;
    const double tu[3] = {1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)};
    const double tv[3] = {2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)};
    for (int r = 0; r < 3; ++r) {
        o.du[r] = (double)R[3 * r] * tu[0] + (double)R[3 * r + 1] * tu[1] + (double)R[3 * r + 2] * tu[2];
        o.dv[r] = (double)R[3 * r] * tv[0] + (double)R[3 * r + 1] * tv[1] + (double)R[3 * r + 2] * tv[2];
        o.Tu[r] = (double)sc[0] * o.du[r];
        o.Tv[r] = (double)sc[1] * o.dv[r];
    }
    const double fx = cam.fx, fy = cam.fy, pz = o.p[2], z2 = pz * pz;
    o.a0 = fx * (o.Tu[0] * pz - o.p[0] * o.Tu[2]) / z2;
    o.a1 = fx * (o.Tv[0] * pz - o.p[0] * o.Tv[2]) / z2;
    o.b0 = fy * (o.Tu[1] * pz - o.p[1] * o.Tu[2]) / z2;
    o.b1 = fy * (o.Tv[1] * pz - o.p[1] * o.Tv[2]) / z2;
    o.c0 = o.Tu[2] / pz;
    o.c1 = o.Tv[2] / pz;
    return o;
}

// SH colour of a primitive at centre mu seen from camera `cam` (clamped at 0)
__device__ __forceinline__ void sh_colour(const ProjectArgs& a, int g, const fh_camera& cam, const float* mu,
                                          float* col) {
    float cp[3];
    cam_centre(cam, cp);
    float dx = mu[0] - cp[0], dy = mu[1] - cp[1], dz = mu[2] - cp[2];
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= il; dy *= il; dz *= il;
    float Y[16];
    sh_basis(a.sh_degree, dx, dy, dz, Y);
    const int nb = (a.sh_degree + 1) * (a.sh_degree + 1);
    const float* shg = a.sh + (size_t)g * nb * 3;
    col[0] = col[1] = col[2] = 0.5f;
    for (int b = 0; b < nb; ++b)
        for (int ch = 0; ch < 3; ++ch) col[ch] += shg[3 * b + ch] * Y[b];
    for (int ch = 0; ch < 3; ++ch) col[ch] = fmaxf(col[ch], 0.0f);
}

// Surfel records, four float4: (x_c hi, y_c hi, x_c lo, y_c lo), (a0, a1, b0,
// b1), (opacity, r, g, b), (D, e1, e2, 0) with D = a0 b1 - a1 b0,
// e1 = a0 c1 - a1 c0, e2 = c0 b1 - c1 b0: for pixel offsets (dx, dy) the ray
// meets the plane at (u, v) = (dx b1 - dy a1, dy a0 - dx b0) / (D - dy e1 - dx e2).
__global__ __launch_bounds__(256) void k_project_surfel(ProjectArgs a, CamTable ct, ViewTable vt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (g >= a.n) return;
    const fh_camera& cam = ct.cam[v];
    const float mu[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
    const float sc[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
    const float4 q4 = reinterpret_cast<const float4*>(a.quats)[g];
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float op = a.opacity[g];
    const BinQ bq = binning_surfel_f32(mu[0], mu[1], mu[2], sc[0], sc[1], q[0], q[1], q[2], q[3], op, cam,
                                       vt.tiles_x[v], vt.tiles_y[v]);
    const size_t j = (size_t)v * a.n + g;
    const bool binned = bq.binned;
    float4 r0 = make_float4(0, 0, 0, 0), r1 = r0, r2 = r0, r3 = r0;
    if (binned) {
        const Srf64 f = srf64(mu, sc, q, cam);
        const double xc = (double)cam.fx * f.p[0] / f.p[2] + (double)cam.cx;
        const double yc = (double)cam.fy * f.p[1] / f.p[2] + (double)cam.cy;
        const double D = f.a0 * f.b1 - f.a1 * f.b0;
        const double e1 = f.a0 * f.c1 - f.a1 * f.c0;
        const double e2 = f.c0 * f.b1 - f.c1 * f.b0;
        const float xh = (float)xc, yh = (float)yc;
        // a non-finite frame keeps its instances but never blends (opacity 0)
        const bool fin = isfinite(D) && isfinite(e1) && isfinite(e2) && isfinite(xc) && isfinite(yc);
        r0 = make_float4(xh, yh, (float)(xc - (double)xh), (float)(yc - (double)yh));
        r1 = make_float4((float)f.a0, (float)f.a1, (float)f.b0, (float)f.b1);
        float col[3];
        sh_colour(a, g, cam, mu, col);
        r2 = make_float4(fin ? op : 0.0f, col[0], col[1], col[2]);
        r3 = make_float4((float)D, (float)e1, (float)e2, 0.0f);
    }
    if (v == 0) {
        bool bad = !(isfinite(op));
        for (int k = 0; k < 3; ++k) bad |= !isfinite(mu[k]) || !isfinite(sc[k]);
        for (int k = 0; k < 4; ++k) bad |= !isfinite(q[k]);
        if (bad) atomicAdd(&a.counters->n_culled_nonfinite, 1ull);
    }
    a.rec[4 * j] = r0;
    a.rec[4 * j + 1] = r1;
    a.rec[4 * j + 2] = r2;
    a.rec[4 * j + 3] = r3;
    a.depth_key[j] = binned ? __float_as_uint(bq.depth) : CULLED_KEY;
    a.rect[j] = binned ? make_int4(bq.x0, bq.y0, bq.x1, bq.y1) : make_int4(0, 0, -1, -1);
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_project(ProjectArgs a, CamTable ct, ViewTable vt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (g >= a.n) return;
    const fh_camera& cam = ct.cam[v];
    const float mu[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
    const float sc[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
    const float4 q4 = reinterpret_cast<const float4*>(a.quats)[g];
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float op = a.opacity[g];
    const BinQ bq = binning_f32(mu[0], mu[1], mu[2], sc[0], sc[1], sc[2], q[0], q[1], q[2], q[3], op, a.bin_rule,
                                cam, vt.tiles_x[v], vt.tiles_y[v]);
    const size_t j = (size_t)v * a.n + g;
    const bool binned = bq.binned;
    float4 r0 = make_float4(0, 0, 0, 0), r1 = r0, r2 = r0;
    if (binned) {
        const Cov64 cv = cov64(mu, sc, q, cam);
        const double det = cv.a * cv.c - cv.b * cv.b;
        const double A = cv.c / det, B = -cv.b / det, C = cv.a / det;
        const double tr = A + C, df = A - C;
        const double disc = sqrt(df * df + 4.0 * B * B);
        const double l1 = 0.5 * (tr + disc);
        const double l2 = (1.0 / det) / l1;
        const double th = 0.5 * atan2(2.0 * B, df);
        const double LOG2E = 1.4426950408889634;
        const double u = (double)cam.fx * cv.p[0] / cv.p[2] + (double)cam.cx;
        const double vv = (double)cam.fy * cv.p[1] / cv.p[2] + (double)cam.cy;
        const float uh = (float)u, vh = (float)vv;
        // a degenerate FP64 covariance keeps its instances but never blends (opacity 0)
        const bool fin = isfinite(det) && det > 0.0 && isfinite(l1) && isfinite(l2) && l2 > 0.0;
        r0 = make_float4(uh, vh, (float)(u - (double)uh), (float)(vv - (double)vh));
        r1 = make_float4((float)cos(th), (float)sin(th), (float)(-0.5 * LOG2E * l1), (float)(-0.5 * LOG2E * l2));
        float col[3];
        sh_colour(a, g, cam, mu, col);
        r2 = make_float4(fin ? op : 0.0f, col[0], col[1], col[2]);
    }
    if (v == 0) {
        bool bad = !(isfinite(op));
        for (int k = 0; k < 3; ++k) bad |= !isfinite(mu[k]) || !isfinite(sc[k]);
        for (int k = 0; k < 4; ++k) bad |= !isfinite(q[k]);
        if (bad) atomicAdd(&a.counters->n_culled_nonfinite, 1ull);
    }
    a.rec[3 * j] = r0;
    a.rec[3 * j + 1] = r1;
    a.rec[3 * j + 2] = r2;
    a.depth_key[j] = binned ? __float_as_uint(bq.depth) : CULLED_KEY;
    a.rect[j] = binned ? make_int4(bq.x0, bq.y0, bq.x1, bq.y1) : make_int4(0, 0, -1, -1);
}

// ---------------------------------------------------------------------------
// Pieces of the projection adjoint shared by both primitives.

// R_q(qn) with qn = q / |q|: upR (adjoint of R_q) -> gq (adjoint of q)
__device__ __forceinline__ void quat_adjoint(const double* qn, double qnorm, const float (*upR)[3], float* gq) {
    const float w = (float)qn[0], x = (float)qn[1], y = (float)qn[2], z = (float)qn[3];
    const float gw = 2.0f * (-z * upR[0][1] + y * upR[0][2] + z * upR[1][0] - x * upR[1][2] - y * upR[2][0] + x * upR[2][1]);
    const float gx = 2.0f * (y * upR[0][1] + z * upR[0][2] + y * upR[1][0] - 2.0f * x * upR[1][1] - w * upR[1][2]
                             + z * upR[2][0] + w * upR[2][1] - 2.0f * x * upR[2][2]);
    const float gy = 2.0f * (-2.0f * y * upR[0][0] + x * upR[0][1] + w * upR[0][2] + x * upR[1][0] + z * upR[1][2]
                             - w * upR[2][0] + z * upR[2][1] - 2.0f * y * upR[2][2]);
    const float gz = 2.0f * (-2.0f * z * upR[0][0] - w * upR[0][1] + x * upR[0][2] + w * upR[1][0] - 2.0f * z * upR[1][1]
                             + y * upR[1][2] + x * upR[2][0] + y * upR[2][1]);
    // qn = q / |q|
    const float dotq = w * gw + x * gx + y * gy + z * gz;
    const float iq = (float)(1.0 / qnorm);
    gq[0] += (gw - w * dotq) * iq;
    gq[1] += (gx - x * dotq) * iq;
    gq[2] += (gy - y * dotq) * iq;
    gq[3] += (gz - z * dotq) * iq;
}

// colour: rgb = max(0, sum_b sh_b Y_b(dir) + 1/2), dir = (mu - cam) / |mu - cam|;
// urgb_in: the view's adjoint of rgb
__device__ __forceinline__ void colour_adjoint(const ProjectBwdArgs& a, const fh_camera& cam, const float* mu,
                                               const float* shg, int nb, const float* urgb_in, float* gmu,
                                               float (*gsh)[3]) {
    float cp[3];
    cam_centre(cam, cp);
    float ddx = mu[0] - cp[0], ddy = mu[1] - cp[1], ddz = mu[2] - cp[2];
    const float il = 1.0f / sqrtf(ddx * ddx + ddy * ddy + ddz * ddz);
    const float dx = ddx * il, dy = ddy * il, dz = ddz * il;
    float Y[16];
    sh_basis(a.sh_degree, dx, dy, dz, Y);
    float raw[3] = {0.5f, 0.5f, 0.5f};
    for (int b = 0; b < nb; ++b)
        for (int ch = 0; ch < 3; ++ch) raw[ch] += shg[3 * b + ch] * Y[b];
    float urgb[3];
    for (int ch = 0; ch < 3; ++ch) urgb[ch] = raw[ch] > 0.0f ? urgb_in[ch] : 0.0f;
    for (int b = 0; b < nb; ++b)
        for (int ch = 0; ch < 3; ++ch) gsh[b][ch] += Y[b] * urgb[ch];
    if (a.sh_degree > 0) {
        float GY[16][3];
        sh_basis_grad(a.sh_degree, dx, dy, dz, GY);
        float udir[3] = {0, 0, 0};
        for (int b = 1; b < nb; ++b) {
            const float s = shg[3 * b] * urgb[0] + shg[3 * b + 1] * urgb[1] + shg[3 * b + 2] * urgb[2];
            udir[0] += GY[b][0] * s;
            udir[1] += GY[b][1] * s;
            udir[2] += GY[b][2] * s;
        }
        const float dd = dx * udir[0] + dy * udir[1] + dz * udir[2];
        gmu[0] += (udir[0] - dx * dd) * il;
        gmu[1] += (udir[1] - dy * dd) * il;
        gmu[2] += (udir[2] - dz * dd) * il;
    }
}

__device__ __forceinline__ void store_grads(const ProjectBwdArgs& a, int g, int nb, const float* gmu, const float* gs,
                                            const float* gq, float gop, const float (*gsh)[3]) {
    for (int k = 0; k < 3; ++k) {
        a.g_means[3 * g + k] = gmu[k];
        a.g_scales[3 * g + k] = gs[k];
    }
    reinterpret_cast<float4*>(a.g_quats)[g] = make_float4(gq[0], gq[1], gq[2], gq[3]);
    a.g_opacity[g] = gop;
    float* gsho = a.g_sh + (size_t)g * nb * 3;
    if (nb == 16) {
        // 48 floats per Gaussian (192 B, 16-B aligned): as twelve float4
        const float* f = &gsh[0][0];
        float4* o4 = reinterpret_cast<float4*>(gsho);
#pragma unroll
        for (int k = 0; k < 12; ++k) o4[k] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
    } else {
        for (int b = 0; b < nb; ++b)
            for (int ch = 0; ch < 3; ++ch) gsho[3 * b + ch] = gsh[b][ch];
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the projection, summed over views in view order (deterministic).
// grad2d[(v*N + g)*12 + k], k: 0 u, 1 v, 2 A, 3 B, 4 C, 5 sum dL/dpower,
// 6..8 rgb, 9 sum w.

template <int GP = 12>
__device__ __forceinline__ bool upstream_zero(const float* grad2d, size_t j) {
    const float4* g4 = reinterpret_cast<const float4*>(grad2d + j * GP);
    bool z = true;
#pragma unroll
    for (int k = 0; k < GP / 4; ++k) {
        const float4 q = g4[k];
        z = z && q.x == 0.f && q.y == 0.f && q.z == 0.f && q.w == 0.f;
    }
    return z;
}

// The outputs are zero-filled before the launch; a Gaussian whose views all
// pass zero upstream terms (no visited instance reached it) keeps them: every
// chained term would be zero.
__global__ __launch_bounds__(256) void k_project_bwd(ProjectBwdArgs a, CamTable ct, int n_views) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    // after an overflow the per-(view, Gaussian) adjoints were not recomputed
    // (they hold an earlier call's values): leave the gradients zero
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    bool any = false;
    for (int v = 0; v < n_views && !any; ++v) {
        const size_t j = (size_t)v * a.n + g;
        any = a.depth_key[j] != CULLED_KEY && !upstream_zero(a.grad2d, j);
    }
    if (!any) return;
    const float mu[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
    const float sc[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
    const float4 q4 = reinterpret_cast<const float4*>(a.quats)[g];
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float op = a.opacity[g];
    const int nb = (a.sh_degree + 1) * (a.sh_degree + 1);
    const float* shg = a.sh + (size_t)g * nb * 3;

    float gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = 0.0f;
    float gsh[16][3];
    for (int b = 0; b < 16; ++b) gsh[b][0] = gsh[b][1] = gsh[b][2] = 0.0f;

    for (int v = 0; v < n_views; ++v) {
        const size_t j = (size_t)v * a.n + g;
        // (a view that no visited instance of this Gaussian reached passes zero
        // upstream terms: every chained term below is then zero)
        if (a.depth_key[j] == CULLED_KEY || upstream_zero(a.grad2d, j)) continue;
        const float* g2 = a.grad2d + j * 12;
        const fh_camera& cam = ct.cam[v];
        const Cov64 cv = cov64(mu, sc, q, cam);

        // opacity: alpha = o G, so dL/do = (sum_p dL/dpower) / o
        gop += g2[5] / op;

        // conic (A, B, C) = (c, -b, a)/det  ->  Sigma2 entries (a, b, c), FP64
        const double a_ = cv.a, b_ = cv.b, c_ = cv.c;
        const double det = a_ * c_ - b_ * b_;
        const double d2 = det * det;
        const double uA = g2[2], uB = g2[3], uC = g2[4];
        const double up_a = (-c_ * c_ * uA + b_ * c_ * uB - b_ * b_ * uC) / d2;
        const double up_b = (2.0 * b_ * c_ * uA - (a_ * c_ + b_ * b_) * uB + 2.0 * a_ * b_ * uC) / d2;
        const double up_c = (-b_ * b_ * uA + a_ * b_ * uB - a_ * a_ * uC) / d2;

        // a = |W0|^2, b = W0 . W1, c = |W1|^2 with W = T M (2x3)
        float upW[2][3];
        for (int l = 0; l < 3; ++l) {
            upW[0][l] = (float)(2.0 * up_a * cv.W[0][l] + up_b * cv.W[1][l]);
            upW[1][l] = (float)(up_b * cv.W[0][l] + 2.0 * up_c * cv.W[1][l]);
        }
        // W = T M: dT = dW M^T, dM = T^T dW
        float upT[2][3], upM[3][3];
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 3; ++k)
                upT[r][k] = upW[r][0] * (float)cv.M[k][0] + upW[r][1] * (float)cv.M[k][1] + upW[r][2] * (float)cv.M[k][2];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) upM[k][l] = (float)cv.T[0][k] * upW[0][l] + (float)cv.T[1][k] * upW[1][l];

        // T = J R_c
        const float* R = cam.R;
        const float uJ00 = upT[0][0] * R[0] + upT[0][1] * R[1] + upT[0][2] * R[2];
        const float uJ02 = upT[0][0] * R[6] + upT[0][1] * R[7] + upT[0][2] * R[8];
        const float uJ11 = upT[1][0] * R[3] + upT[1][1] * R[4] + upT[1][2] * R[5];
        const float uJ12 = upT[1][0] * R[6] + upT[1][1] * R[7] + upT[1][2] * R[8];

        // J, (u, v) -> camera-space centre
        const float px = (float)cv.p[0], py = (float)cv.p[1], pz = (float)cv.p[2];
        const float fx = cam.fx, fy = cam.fy;
        const float iz = 1.0f / pz, iz2 = iz * iz, iz3 = iz2 * iz;
        const float uu = g2[0], uv = g2[1];
        const float upx = fx * iz * uu - fx * iz2 * uJ02;
        const float upy = fy * iz * uv - fy * iz2 * uJ12;
        const float upz = -fx * px * iz2 * uu - fy * py * iz2 * uv - fx * iz2 * uJ00 + 2.0f * fx * px * iz3 * uJ02
                          - fy * iz2 * uJ11 + 2.0f * fy * py * iz3 * uJ12;
        // p = R_c mu + t
        for (int k = 0; k < 3; ++k) gmu[k] += R[k] * upx + R[3 + k] * upy + R[6 + k] * upz;

        // M = R_q diag(s)
        float upR[3][3];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) upR[k][l] = upM[k][l] * sc[l];
        for (int l = 0; l < 3; ++l)
            gs[l] += upM[0][l] * (float)cv.Rq[0][l] + upM[1][l] * (float)cv.Rq[1][l] + upM[2][l] * (float)cv.Rq[2][l];

        quat_adjoint(cv.qn, cv.qnorm, upR, gq);
        colour_adjoint(a, cam, mu, shg, nb, g2 + 6, gmu, gsh);
    }
    store_grads(a, g, nb, gmu, gs, gq, gop, gsh);
}

// Surfel adjoint, views in view order.  grad2d[(v*N + g)*16 + k], k: 0..8
// the record entries (x_c, y_c, a0, a1, b0, b1, D, e1, e2), 9 sum dL/dpower,
// 10..12 rgb, 13 sum w.  The chain in FP64: (D, e1, e2) -> (a, b, c), then
// (x_c, y_c, a, b, c) -> (p, T_u, T_v) -> (mu, s_u, s_v, q).
__global__ __launch_bounds__(256) void k_project_bwd_surfel(ProjectBwdArgs a, CamTable ct, int n_views) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    if (a.counters->inst_overflow || a.counters->visit_overflow) return;
    bool any = false;
    for (int v = 0; v < n_views && !any; ++v) {
        const size_t j = (size_t)v * a.n + g;
        any = a.depth_key[j] != CULLED_KEY && !upstream_zero<16>(a.grad2d, j);
    }
    if (!any) return;
    const float mu[3] = {a.means[3 * g], a.means[3 * g + 1], a.means[3 * g + 2]};
    const float sc[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
    const float4 q4 = reinterpret_cast<const float4*>(a.quats)[g];
    const float q[4] = {q4.x, q4.y, q4.z, q4.w};
    const float op = a.opacity[g];
    const int nb = (a.sh_degree + 1) * (a.sh_degree + 1);
    const float* shg = a.sh + (size_t)g * nb * 3;
    float gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = 0.0f;
    float gsh[16][3];
    for (int b = 0; b < 16; ++b) gsh[b][0] = gsh[b][1] = gsh[b][2] = 0.0f;
    for (int v = 0; v < n_views; ++v) {
        const size_t j = (size_t)v * a.n + g;
        if (a.depth_key[j] == CULLED_KEY || upstream_zero<16>(a.grad2d, j)) continue;
        const float* g2 = a.grad2d + j * 16;
        const fh_camera& cam = ct.cam[v];
        const Srf64 f = srf64(mu, sc, q, cam);
        gop += g2[9] / op;
        // (D, e1, e2) -> (a, b, c)
        const double gD = g2[6], ge1 = g2[7], ge2 = g2[8];
        const double ga0 = g2[2] + f.b1 * gD + f.c1 * ge1;
        const double ga1 = g2[3] - f.b0 * gD - f.c0 * ge1;
        const double gb0 = g2[4] - f.a1 * gD - f.c1 * ge2;
        const double gb1 = g2[5] + f.a0 * gD + f.c0 * ge2;
        const double gc0 = -f.a1 * ge1 + f.b1 * ge2;
        const double gc1 = f.a0 * ge1 - f.b0 * ge2;
        // (x_c, y_c, a, b, c) -> (p, T_u, T_v)
        const double fx = cam.fx, fy = cam.fy, px = f.p[0], py = f.p[1], z = f.p[2];
        const double z2 = z * z, z3 = z2 * z;
        const double gxc = g2[0], gyc = g2[1];
        double gp[3] = {fx / z * gxc, fy / z * gyc, -fx * px / z2 * gxc - fy * py / z2 * gyc};
        double gT[2][3];
        const double* Ts[2] = {f.Tu, f.Tv};
        const double gas[2] = {ga0, ga1}, gbs[2] = {gb0, gb1}, gcs[2] = {gc0, gc1};
        for (int i = 0; i < 2; ++i) {
            const double* T = Ts[i];
            gT[i][0] = fx / z * gas[i];
            gT[i][1] = fy / z * gbs[i];
            gT[i][2] = -fx * px / z2 * gas[i] - fy * py / z2 * gbs[i] + gcs[i] / z;
            gp[0] += -fx * T[2] / z2 * gas[i];
            gp[1] += -fy * T[2] / z2 * gbs[i];
            gp[2] += (-fx * T[0] / z2 + 2.0 * fx * px * T[2] / z3) * gas[i] +
                     (-fy * T[1] / z2 + 2.0 * fy * py * T[2] / z3) * gbs[i] - T[2] / z2 * gcs[i];
        }
        // p = R_c mu + t
        const float* R = cam.R;
        for (int k = 0; k < 3; ++k) gmu[k] += (float)((double)R[k] * gp[0] + (double)R[3 + k] * gp[1] + (double)R[6 + k] * gp[2]);
        // T_u = s_u R_c t_u, T_v = s_v R_c t_v
        gs[0] += (float)(gT[0][0] * f.du[0] + gT[0][1] * f.du[1] + gT[0][2] * f.du[2]);
        gs[1] += (float)(gT[1][0] * f.dv[0] + gT[1][1] * f.dv[1] + gT[1][2] * f.dv[2]);
        float upR[3][3];
        for (int k = 0; k < 3; ++k) {
            upR[k][0] = (float)(((double)R[k] * gT[0][0] + (double)R[3 + k] * gT[0][1] + (double)R[6 + k] * gT[0][2]) * sc[0]);
            upR[k][1] = (float)(((double)R[k] * gT[1][0] + (double)R[3 + k] * gT[1][1] + (double)R[6 + k] * gT[1][2]) * sc[1]);
            upR[k][2] = 0.0f;
        }
        quat_adjoint(f.qn, f.qnorm, upR, gq);
        colour_adjoint(a, cam, mu, shg, nb, g2 + 10, gmu, gsh);
    }
    store_grads(a, g, nb, gmu, gs, gq, gop, gsh);
}

// ---------------------------------------------------------------------------
void launch_project(const ProjectArgs& a, const CamTable& ct, const ViewTable& vt, int n_views, hipStream_t s) {
    dim3 grid((a.n + 255) / 256, n_views);
    if (a.prim == FH_PRIM_SURFEL)
        hipLaunchKernelGGL(k_project_surfel, grid, dim3(256), 0, s, a, ct, vt);
    else
        hipLaunchKernelGGL(k_project, grid, dim3(256), 0, s, a, ct, vt);
}

void launch_project_bwd(const ProjectBwdArgs& a, const CamTable& ct, int n_views, hipStream_t s) {
    const int64_t nsh = (int64_t)(a.sh_degree + 1) * (a.sh_degree + 1) * 3;
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.g_means), (int64_t)a.n * 3, 0u, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.g_scales), (int64_t)a.n * 3, 0u, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.g_quats), (int64_t)a.n * 4, 0u, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.g_opacity), (int64_t)a.n, 0u, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.g_sh), (int64_t)a.n * nsh, 0u, s);
    if (a.prim == FH_PRIM_SURFEL)
        hipLaunchKernelGGL(k_project_bwd_surfel, dim3((a.n + 255) / 256), dim3(256), 0, s, a, ct, n_views);
    else
        hipLaunchKernelGGL(k_project_bwd, dim3((a.n + 255) / 256), dim3(256), 0, s, a, ct, n_views);
}

}  // namespace fh
