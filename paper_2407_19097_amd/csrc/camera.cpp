// Host-side camera composition: the only FP64 arithmetic of the library.
//
// The paper renders training views with a 60 degree field of view and near /
// far planes at 0.1 / 2e5 (Sec. 3.3).  The clip matrix is M = P * V with V a
// right-handed look-at and P the OpenGL perspective with aspect W/H.  Rows
// are written out in closed form (P is sparse), evaluated in double and
// rounded once per entry to float.
#include <cmath>

#include "narvis.h"

namespace {

struct Vec3 {
    double x, y, z;
};

Vec3 sub(const double a[3], const double b[3]) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
double dot(const Vec3 &a, const Vec3 &b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
Vec3 cross(const Vec3 &a, const Vec3 &b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

bool finite3(const double v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

}  // namespace

extern "C" narvis_status narvis_camera_matrix(const narvis_camera *cam, int32_t W, int32_t H,
                                              float vp[16], float *near_f, float *far_f)
{
    if (!cam || !vp || W < 1 || H < 1) return NARVIS_ERR_INVALID_ARG;
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up)) return NARVIS_ERR_INVALID_ARG;
    if (!(cam->fovy_deg > 0.0 && cam->fovy_deg < 180.0)) return NARVIS_ERR_INVALID_ARG;
    if (!(cam->znear > 0.0 && cam->znear < cam->zfar && std::isfinite(cam->zfar))) return NARVIS_ERR_INVALID_ARG;

    Vec3 f = sub(cam->target, cam->eye);
    double fl = std::sqrt(dot(f, f));
    if (!(fl > 0.0)) return NARVIS_ERR_INVALID_ARG;
    f = {(cam->target[0] - cam->eye[0]) / fl, (cam->target[1] - cam->eye[1]) / fl,
         (cam->target[2] - cam->eye[2]) / fl};
    Vec3 up = {cam->up[0], cam->up[1], cam->up[2]};
    Vec3 s = cross(f, up);
    double sl = std::sqrt(dot(s, s));
    if (!(sl > 1e-12)) return NARVIS_ERR_INVALID_ARG;
    s = {s.x / sl, s.y / sl, s.z / sl};
    Vec3 u = cross(s, f);
    Vec3 eye = {cam->eye[0], cam->eye[1], cam->eye[2]};

    const double kPi = 3.14159265358979323846;
    double t = std::tan(cam->fovy_deg * (kPi / 180.0) / 2.0);
    double aspect = (double)W / (double)H;
    double p00 = 1.0 / (aspect * t);
    double p11 = 1.0 / t;
    double n = cam->znear, fa = cam->zfar;
    double A = -(fa + n) / (fa - n);
    double B = -2.0 * fa * n / (fa - n);

    double M[16] = {
        p00 * s.x, p00 * s.y, p00 * s.z, p00 * (-dot(s, eye)),
        p11 * u.x, p11 * u.y, p11 * u.z, p11 * (-dot(u, eye)),
        A * -f.x,  A * -f.y,  A * -f.z,  A * dot(f, eye) + B,
        f.x,       f.y,       f.z,       -dot(f, eye),
    };
    // the zero terms of the matrix product P * V add +0.0, which turns a
    // negative zero into a positive one; do the same so exact zeros agree
    for (int k = 0; k < 16; ++k) vp[k] = (float)(M[k] + 0.0);
    if (near_f) *near_f = (float)n;
    if (far_f) *far_f = (float)fa;
    return NARVIS_OK;
}

extern "C" narvis_status narvis_camera_focal_px(const narvis_camera *cam, int32_t H, float *focal_px)
{
    if (!cam || !focal_px || H < 1) return NARVIS_ERR_INVALID_ARG;
    if (!(cam->fovy_deg > 0.0 && cam->fovy_deg < 180.0)) return NARVIS_ERR_INVALID_ARG;
    const double kPi = 3.14159265358979323846;
    const double t = std::tan(cam->fovy_deg * (kPi / 180.0) / 2.0);
    *focal_px = (float)((double)H * 0.5 / t);
    return NARVIS_OK;
}
