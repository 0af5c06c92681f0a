// Reprojection of a 3-D point by a 9-parameter camera and its analytic Jacobian
// (Sec. 3: f(x) and J = [J_c, J_p]).  Always evaluated in FP64.
//
// Camera c = (w, t, f, k1, k2): P = R(w) X + t with the Rodrigues rotation
// R = I + a [w]x + b [w]x^2 (a = sin th / th, b = (1 - cos th) / th^2),
// (x, y) = (P_x, P_y) / P_z, r2 = x^2 + y^2, pixel = f (1 + k1 r2 + k2 r2^2) (x, y).
// dP/dw = -R [X]x J_r(w), with the right Jacobian of SO(3)
// J_r = I - b [w]x + c [w]x^2, c = (th - sin th) / th^3.
#pragma once
#include <hip/hip_runtime.h>

namespace stba {

struct RodCoef {
    double a, b, c;
};

__device__ inline RodCoef rodrigues_coefficients(double th2) {
    RodCoef r;
    if (th2 < 1e-8) {
        r.a = 1.0 - th2 / 6.0;
        r.b = 0.5 - th2 / 24.0;
        r.c = 1.0 / 6.0 - th2 / 120.0;
    } else {
        const double th = sqrt(th2);
        double s, co;
        sincos(th, &s, &co);
        r.a = s / th;
        r.b = (1.0 - co) / th2;
        r.c = (th - s) / (th2 * th);
    }
    return r;
}

// R = I + a K + b K^2 with K = [w]x, using K^2 = w w^T - th2 I.
__device__ inline void rotation_from_vector(const double w[3], double th2, const RodCoef &k, double R[3][3]) {
    const double a = k.a, b = k.b;
    R[0][0] = 1.0 + b * (w[0] * w[0] - th2);
    R[0][1] = -a * w[2] + b * w[0] * w[1];
    R[0][2] = a * w[1] + b * w[0] * w[2];
    R[1][0] = a * w[2] + b * w[1] * w[0];
    R[1][1] = 1.0 + b * (w[1] * w[1] - th2);
    R[1][2] = -a * w[0] + b * w[1] * w[2];
    R[2][0] = -a * w[1] + b * w[2] * w[0];
    R[2][1] = a * w[0] + b * w[2] * w[1];
    R[2][2] = 1.0 + b * (w[2] * w[2] - th2);
}


// The camera's part of the projection, independent of the point: R(w) (row-
// major, 9), the right Jacobian J_r(w) (row-major, 9), t (3), f, k1, k2: 24
// doubles, formed once per camera where many observations share it.
constexpr int kCamPre = 24;

__device__ inline void camera_pre(const double c[9], double cp[kCamPre]) {
    const double w[3] = {c[0], c[1], c[2]};
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const RodCoef k = rodrigues_coefficients(th2);
    double R[3][3];
    rotation_from_vector(w, th2, k, R);
    // J_r = I - b K + c K^2 = (1 - c th2) I - b K + c w w^T
    const double bb = k.b, cc = k.c;
    double Jr[3][3];
    Jr[0][0] = 1.0 + cc * (w[0] * w[0] - th2);
    Jr[0][1] = bb * w[2] + cc * w[0] * w[1];
    Jr[0][2] = -bb * w[1] + cc * w[0] * w[2];
    Jr[1][0] = -bb * w[2] + cc * w[1] * w[0];
    Jr[1][1] = 1.0 + cc * (w[1] * w[1] - th2);
    Jr[1][2] = bb * w[0] + cc * w[1] * w[2];
    Jr[2][0] = bb * w[1] + cc * w[2] * w[0];
    Jr[2][1] = -bb * w[0] + cc * w[2] * w[1];
    Jr[2][2] = 1.0 + cc * (w[2] * w[2] - th2);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cp[3 * i + j] = R[i][j];
            cp[9 + 3 * i + j] = Jr[i][j];
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) cp[18 + i] = c[3 + i];
}

// Pixel of point X from the camera's part cp: the same operations as the
// pixel of project_jac_pre, so residuals with and without the Jacobian agree
// bit for bit.
__device__ inline void project_pre(const double cp[kCamPre], const double X[3], double pix[2]) {
    const double *R = cp;
    double P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + cp[18 + i];
    const double iz = 1.0 / P[2];
    const double x = P[0] * iz, y = P[1] * iz;
    const double fl = cp[21], k1 = cp[22], k2 = cp[23];
    const double r2 = x * x + y * y;
    const double d = 1.0 + k1 * r2 + k2 * r2 * r2;
    pix[0] = fl * d * x;
    pix[1] = fl * d * y;
}

// Pixel of point X in camera c.
__device__ inline void camera_project(const double c[9], const double X[3], double pix[2]) {
    double cp[kCamPre];
    camera_pre(c, cp);
    project_pre(cp, X, pix);
}

// Pixel plus Jacobian blocks Jc [2][9] and Jp [2][3] (row-major) from the
// camera's part cp and the point X.
__device__ inline void project_jac_pre(const double cp[kCamPre], const double X[3], double pix[2], double Jc[2][9],
                                       double Jp[2][3]) {
    const double *R = cp, *Jr = cp + 9;
    double P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + cp[18 + i];
    const double iz = 1.0 / P[2];
    const double x = P[0] * iz, y = P[1] * iz;
    const double fl = cp[21], k1 = cp[22], k2 = cp[23];
    const double r2 = x * x + y * y;
    const double d = 1.0 + k1 * r2 + k2 * r2 * r2;
    pix[0] = fl * d * x;
    pix[1] = fl * d * y;
    // d pixel / d (x, y) = f [d I + 2 s (x, y)^T (x, y)], s = k1 + 2 k2 r2
    const double s = k1 + 2.0 * k2 * r2;
    const double A00 = fl * (d + 2.0 * s * x * x), A01 = fl * (2.0 * s * x * y);
    const double A11 = fl * (d + 2.0 * s * y * y);
    // d pixel / d P = A * (1/P_z) [[1, 0, -x], [0, 1, -y]]
    double B[2][3];
    B[0][0] = A00 * iz;
    B[0][1] = A01 * iz;
    B[0][2] = -(A00 * x + A01 * y) * iz;
    B[1][0] = A01 * iz;
    B[1][1] = A11 * iz;
    B[1][2] = -(A01 * x + A11 * y) * iz;
    // [X]x J_r
    double XJ[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        XJ[0][j] = -X[2] * Jr[3 + j] + X[1] * Jr[6 + j];
        XJ[1][j] = X[2] * Jr[j] - X[0] * Jr[6 + j];
        XJ[2][j] = -X[1] * Jr[j] + X[0] * Jr[3 + j];
    }
    // dP/dw = -R [X]x J_r
    double dPdw[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            dPdw[i][j] = -(R[3 * i] * XJ[0][j] + R[3 * i + 1] * XJ[1][j] + R[3 * i + 2] * XJ[2][j]);
    const double xy[2] = {x, y};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Jc[i][j] = B[i][0] * dPdw[0][j] + B[i][1] * dPdw[1][j] + B[i][2] * dPdw[2][j];
            Jc[i][3 + j] = B[i][j];
            Jp[i][j] = B[i][0] * R[j] + B[i][1] * R[3 + j] + B[i][2] * R[6 + j];
        }
        Jc[i][6] = d * xy[i];
        Jc[i][7] = fl * r2 * xy[i];
        Jc[i][8] = fl * r2 * r2 * xy[i];
    }
}

// Pixel plus Jacobian blocks Jc [2][9] and Jp [2][3] (row-major).
__device__ inline void camera_project_jac(const double c[9], const double X[3], double pix[2],
                                          double Jc[2][9], double Jp[2][3]) {
    double cp[kCamPre];
    camera_pre(c, cp);
    project_jac_pre(cp, X, pix, Jc, Jp);
}

// Robust loss (Sec. 5.1): Huber with scale a on s = ||f_o||^2, rho(s) = s up to
// a^2 and 2 a sqrt(s) - a^2 above; the IRLS weight on f and J is sqrt(rho'(s)),
// rho'(s) = a / sqrt(s) above a^2.  a = 0: the squared loss.
__device__ inline double huber_rho(double s, double a) { return (a > 0.0 && s > a * a) ? 2.0 * a * sqrt(s) - a * a : s; }
__device__ inline double huber_root_weight(double s, double a) {
    return (a > 0.0 && s > a * a) ? sqrt(a / sqrt(s)) : 1.0;
}

}  // namespace stba
