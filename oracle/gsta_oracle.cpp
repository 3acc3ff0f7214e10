// FP64 CPU oracle of the GSta rasterizer path -- TEST INFRASTRUCTURE ONLY.
//
// This file is the plain, slow reference that the GPU library is checked
// against.  Only the test-suite, the smoke check and the CPU-baseline leg of
// the benchmark load it.  It shares no code, header or constant table with
// the GPU library.
//
// What it computes (paper: "GSta: Efficient Training Scheme with Siestaed
// Gaussians for Monocular 3D Scene Reconstruction", arXiv 2504.06716):
//   * Section 3.1: a Gaussian is a mean, a scale and a rotation quaternion
//     (covariance R S S^T R^T), an opacity and SH colour coefficients up to
//     3 bands; it is projected to a 2-D Gaussian (eq. 1, EWA splatting) and
//     pixels blend the sorted Gaussians front to back (eq. 2).
//   * Section 3.2.4: the backward pass produces per-Gaussian gradients and
//     skips Gaussians whose freeze flag is set.
// Conventions the paper leaves open (near plane 0.2, 2-D dilation 0.3, 3-sigma
// ellipse, alpha floor 1/255, alpha cap 0.99, transmittance floor 1e-4,
// tangent clamp 1.3) are the Gaussian-splatting conventions; each is written
// out where it is used.
//
// Every value is double precision.  The only deliberate float rounding is the
// depth sort key, which is the float32 value of the camera-space depth, so
// that both implementations order Gaussians by the same key.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;
const double kNear = 0.2;          // cull when camera-space depth <= 0.2
const double kDilate = 0.3;        // added to the diagonal of the 2-D covariance
const double kTanClamp = 1.3;      // tangent-plane clamp factor used inside J only
const double kPowerFloor = -4.5;   // 3-sigma ellipse: -0.5 * 3^2
const double kAlphaMin = 1.0 / 255.0;
const double kAlphaMax = 0.99;
const double kTMin = 1e-4;
const double kInf = std::numeric_limits<double>::infinity();

struct Cam {
    int W, H;
    double fx, fy, cx, cy;
    double R[3][3];
    double t[3];
    double pos[3];
    double near;
};

Cam read_cam(const double* c) {
    Cam k;
    k.W = (int)c[0];
    k.H = (int)c[1];
    k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) k.R[i][j] = c[6 + 4 * i + j];
        k.t[i] = c[6 + 4 * i + 3];
    }
    for (int i = 0; i < 3; ++i) k.pos[i] = c[18 + i];
    k.near = c[21];
    return k;
}

// ---------------------------------------------------------------------------
// Real spherical harmonics (Section 3.1: colour from up to 3 SH bands).
// B_k with k = l*l + l + m is a homogeneous polynomial of degree l in the unit
// direction (x, y, z), scaled to unit L2 norm on the sphere, positive sign.
// ---------------------------------------------------------------------------
struct ShConst {
    double c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
    ShConst() {
        c0 = 1.0 / (2.0 * std::sqrt(kPi));
        c1 = std::sqrt(3.0 / (4.0 * kPi));
        c2a = std::sqrt(15.0 / (4.0 * kPi));
        c2b = std::sqrt(5.0 / (16.0 * kPi));
        c2c = std::sqrt(15.0 / (16.0 * kPi));
        c3a = std::sqrt(35.0 / (32.0 * kPi));
        c3b = std::sqrt(105.0 / (4.0 * kPi));
        c3c = std::sqrt(21.0 / (32.0 * kPi));
        c3d = std::sqrt(7.0 / (16.0 * kPi));
        c3e = std::sqrt(105.0 / (16.0 * kPi));
    }
};
const ShConst SH;

// B[k] for k < (degree+1)^2, and dB[k][0..2] = dB_k / d(x, y, z).
void sh_basis(int degree, double x, double y, double z, double* B, double (*dB)[3]) {
    double b[16], d[16][3];
    for (int k = 0; k < 16; ++k) { b[k] = 0; d[k][0] = d[k][1] = d[k][2] = 0; }
    b[0] = SH.c0;
    if (degree >= 1) {
        b[1] = SH.c1 * y; d[1][1] = SH.c1;
        b[2] = SH.c1 * z; d[2][2] = SH.c1;
        b[3] = SH.c1 * x; d[3][0] = SH.c1;
    }
    if (degree >= 2) {
        b[4] = SH.c2a * x * y;  d[4][0] = SH.c2a * y;  d[4][1] = SH.c2a * x;
        b[5] = SH.c2a * y * z;  d[5][1] = SH.c2a * z;  d[5][2] = SH.c2a * y;
        b[6] = SH.c2b * (2 * z * z - x * x - y * y);
        d[6][0] = -2 * SH.c2b * x; d[6][1] = -2 * SH.c2b * y; d[6][2] = 4 * SH.c2b * z;
        b[7] = SH.c2a * x * z;  d[7][0] = SH.c2a * z;  d[7][2] = SH.c2a * x;
        b[8] = SH.c2c * (x * x - y * y);
        d[8][0] = 2 * SH.c2c * x; d[8][1] = -2 * SH.c2c * y;
    }
    if (degree >= 3) {
        b[9] = SH.c3a * y * (3 * x * x - y * y);
        d[9][0] = SH.c3a * 6 * x * y; d[9][1] = SH.c3a * (3 * x * x - 3 * y * y);
        b[10] = SH.c3b * x * y * z;
        d[10][0] = SH.c3b * y * z; d[10][1] = SH.c3b * x * z; d[10][2] = SH.c3b * x * y;
        b[11] = SH.c3c * y * (4 * z * z - x * x - y * y);
        d[11][0] = SH.c3c * (-2 * x * y); d[11][1] = SH.c3c * (4 * z * z - x * x - 3 * y * y);
        d[11][2] = SH.c3c * 8 * y * z;
        b[12] = SH.c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
        d[12][0] = SH.c3d * (-6 * x * z); d[12][1] = SH.c3d * (-6 * y * z);
        d[12][2] = SH.c3d * (6 * z * z - 3 * x * x - 3 * y * y);
        b[13] = SH.c3c * x * (4 * z * z - x * x - y * y);
        d[13][0] = SH.c3c * (4 * z * z - 3 * x * x - y * y); d[13][1] = SH.c3c * (-2 * x * y);
        d[13][2] = SH.c3c * 8 * x * z;
        b[14] = SH.c3e * z * (x * x - y * y);
        d[14][0] = SH.c3e * 2 * x * z; d[14][1] = SH.c3e * (-2 * y * z);
        d[14][2] = SH.c3e * (x * x - y * y);
        b[15] = SH.c3a * x * (x * x - 3 * y * y);
        d[15][0] = SH.c3a * (3 * x * x - 3 * y * y); d[15][1] = SH.c3a * (-6 * x * y);
    }
    int K = (degree + 1) * (degree + 1);
    for (int k = 0; k < K; ++k) {
        B[k] = b[k];
        if (dB) for (int a = 0; a < 3; ++a) dB[k][a] = d[k][a];
    }
}

// ---------------------------------------------------------------------------
// Projection of one Gaussian (Section 3.1, eq. 1 and the EWA splatting it
// cites): covariance, 2-D covariance, conic, screen mean, tile rectangle,
// SH colour and opacity.  Everything the backward needs is kept.
// ---------------------------------------------------------------------------
struct Proj {
    bool visible;
    double mu[3], xc[3];
    double s[3], qn[4], qnorm, Rq[3][3], M[3][3], Sigma[3][3];
    double rx, ry, rxc, ryc, limx, limy;
    bool clx, cly;
    double J[2][3], T[2][3];
    double a, b, c, det, conic[3];
    double u, v, z;
    float z32;
    double ex, ey;
    int tx0, tx1, ty0, ty1;
    double dir[3], dlen, dn[3];
    double B[16];
    double raw[3], rgb[3];
    bool clamped[3];
    double opacity;
    double m_near, m_det, m_rect, m_tan, m_col;
};

// Opacity activation (Section 4.1): 0 sigmoid of the logit in row 10; 1 the
// absolute value of row 10, used by the finetune stage.
int g_opacity_act = 0;

// SH-band masking (Section 3.3; learned only in the finetune stage): three
// mask logits per Gaussian, one per SH band l = 1..3 (row l - 1 of a [3][ld]
// block).  The forward uses the hard gate M_l = 1 if sigmoid(logit) > the
// threshold, else 0, as a factor on every coefficient of band l (band 0 is
// never masked); the backward takes the straight-through estimate
// dL/dlogit = dL/dM_l sigmoid'(logit).  Off (nullptr) by default.
const double* g_shm = nullptr;
int64_t g_shm_ld = 0;
double g_shm_threshold = 0.0;
double* g_shm_grad = nullptr;      // [3][ld] output of the backward, or nullptr

int sh_band(int k) { return k < 1 ? 0 : (k < 4 ? 1 : (k < 9 ? 2 : 3)); }

double sigmoid(double x) { return 1.0 / (1.0 + std::exp(-x)); }

// Gate of band l of Gaussian g.  sigmoid(logit) > t is the same test as
// logit > ln(t / (1 - t)); the decision is taken in the rasterizer's
// precision, the float32 logit against the float32-rounded threshold logit.
double band_gate(int64_t g, int l) {
    if (!g_shm || l == 0) return 1.0;
    const float x = (float)g_shm[(int64_t)(l - 1) * g_shm_ld + g];
    const float xt = (float)std::log(g_shm_threshold / (1.0 - g_shm_threshold));
    return x > xt ? 1.0 : 0.0;
}

double frac_dist(double x) {   // distance of x to the nearest integer
    return std::fabs(x - std::nearbyint(x));
}

void project(const double* P, int64_t n, int64_t ld, int degree, int64_t g, const Cam& cam,
             int tw, int th, Proj& p) {
    auto par = [&](int row) { return P[(int64_t)row * ld + g]; };
    for (int i = 0; i < 3; ++i) p.mu[i] = par(i);
    for (int i = 0; i < 3; ++i)
        p.xc[i] = cam.R[i][0] * p.mu[0] + cam.R[i][1] * p.mu[1] + cam.R[i][2] * p.mu[2] + cam.t[i];
    p.z = p.xc[2];
    p.z32 = (float)p.z;
    p.m_near = std::fabs(p.z - cam.near) / cam.near;
    p.visible = false;
    p.m_det = p.m_rect = p.m_tan = p.m_col = kInf;
    p.tx0 = p.tx1 = p.ty0 = p.ty1 = 0;

    // Activations (Section 3.1): scale = exp(log-scale); unit quaternion.
    for (int i = 0; i < 3; ++i) p.s[i] = std::exp(par(3 + i));
    double q[4] = {par(6), par(7), par(8), par(9)};
    p.qnorm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) p.qn[i] = q[i] / p.qnorm;
    double w = p.qn[0], x = p.qn[1], y = p.qn[2], zq = p.qn[3];
    double Rq[3][3] = {
        {1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y)},
        {2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x)},
        {2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p.Rq[i][j] = Rq[i][j];
            p.M[i][j] = Rq[i][j] * p.s[j];                   // M = R S
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += p.M[i][k] * p.M[j][k];
            p.Sigma[i][j] = acc;                              // Sigma = M M^T
        }

    // Opacity (sigmoid of the logit, or |x| in the finetune stage) and colour
    // are defined for every Gaussian.
    p.opacity = g_opacity_act ? std::fabs(par(10)) : 1.0 / (1.0 + std::exp(-par(10)));
    for (int i = 0; i < 3; ++i) p.dir[i] = p.mu[i] - cam.pos[i];
    p.dlen = std::sqrt(p.dir[0] * p.dir[0] + p.dir[1] * p.dir[1] + p.dir[2] * p.dir[2]);
    for (int i = 0; i < 3; ++i) p.dn[i] = p.dir[i] / p.dlen;
    sh_basis(degree, p.dn[0], p.dn[1], p.dn[2], p.B, nullptr);
    int K = (degree + 1) * (degree + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0;
        for (int k = 0; k < K; ++k) acc += band_gate(g, sh_band(k)) * par(11 + 3 * k + ch) * p.B[k];
        p.raw[ch] = acc + 0.5;
        p.clamped[ch] = p.raw[ch] < 0;
        p.rgb[ch] = p.clamped[ch] ? 0.0 : p.raw[ch];
        p.m_col = std::min(p.m_col, std::fabs(p.raw[ch]));
    }

    if (!(p.z > cam.near)) return;

    // EWA: J is the Jacobian of the perspective map at the mean; the
    // tangent ratios inside J are clamped to 1.3x the half field of view.
    p.rx = p.xc[0] / p.z;
    p.ry = p.xc[1] / p.z;
    p.limx = kTanClamp * (0.5 * cam.W) / cam.fx;
    p.limy = kTanClamp * (0.5 * cam.H) / cam.fy;
    p.clx = std::fabs(p.rx) > p.limx;
    p.cly = std::fabs(p.ry) > p.limy;
    p.rxc = p.clx ? std::copysign(p.limx, p.rx) : p.rx;
    p.ryc = p.cly ? std::copysign(p.limy, p.ry) : p.ry;
    p.m_tan = std::min(std::fabs(std::fabs(p.rx) - p.limx) / p.limx,
                       std::fabs(std::fabs(p.ry) - p.limy) / p.limy);
    double J[2][3] = {{cam.fx / p.z, 0.0, -cam.fx * p.rxc / p.z},
                      {0.0, cam.fy / p.z, -cam.fy * p.ryc / p.z}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            p.J[i][j] = J[i][j];
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[i][k] * cam.R[k][j];
            p.T[i][j] = acc;                                  // T = J W
        }
    double C2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += p.T[i][k] * p.Sigma[k][l] * p.T[j][l];
            C2[i][j] = acc;                                   // Sigma' = T Sigma T^T
        }
    p.a = C2[0][0] + kDilate;
    p.b = C2[0][1];
    p.c = C2[1][1] + kDilate;
    p.det = p.a * p.c - p.b * p.b;
    p.m_det = p.det / (p.a * p.c);
    if (!(p.det > 0)) return;
    p.conic[0] = p.c / p.det;
    p.conic[1] = -p.b / p.det;
    p.conic[2] = p.a / p.det;
    p.u = cam.fx * p.rx + cam.cx;
    p.v = cam.fy * p.ry + cam.cy;

    // Tile rectangle: tile column t is touched iff the pixel columns
    // [tw*t, tw*t + tw-1] meet [u - ex, u + ex] with ex = 3 sqrt(Sigma'_xx),
    // the exact bounding box of the 3-sigma ellipse (likewise for rows).
    p.ex = 3.0 * std::sqrt(p.a);
    p.ey = 3.0 * std::sqrt(p.c);
    int ntx = (cam.W + tw - 1) / tw, nty = (cam.H + th - 1) / th;
    double fx0 = (p.u - p.ex - (tw - 1)) / tw, fx1 = (p.u + p.ex) / tw;
    double fy0 = (p.v - p.ey - (th - 1)) / th, fy1 = (p.v + p.ey) / th;
    auto clampd = [](double x, double lo, double hi) { return std::min(std::max(x, lo), hi); };
    p.tx0 = (int)clampd(std::ceil(fx0), 0, ntx);
    p.tx1 = (int)clampd(std::floor(fx1) + 1, 0, ntx);
    p.ty0 = (int)clampd(std::ceil(fy0), 0, nty);
    p.ty1 = (int)clampd(std::floor(fy1) + 1, 0, nty);
    double mr = kInf;
    if (fx0 > -1 && fx0 < ntx) mr = std::min(mr, frac_dist(fx0) * tw);
    if (fx1 > -1 && fx1 < ntx) mr = std::min(mr, frac_dist(fx1) * tw);
    if (fy0 > -1 && fy0 < nty) mr = std::min(mr, frac_dist(fy0) * th);
    if (fy1 > -1 && fy1 < nty) mr = std::min(mr, frac_dist(fy1) * th);
    p.m_rect = mr;
    p.visible = (p.tx0 < p.tx1) && (p.ty0 < p.ty1);
}

// Visible Gaussians in ascending (float32 depth, gid) order, the blending
// order of Section 3.1; equal depths keep ascending gid (stable sort).
std::vector<int64_t> depth_order(const std::vector<Proj>& pr) {
    std::vector<int64_t> ids;
    for (int64_t g = 0; g < (int64_t)pr.size(); ++g)
        if (pr[g].visible) ids.push_back(g);
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int64_t x, int64_t y) { return pr[x].z32 < pr[y].z32; });
    return ids;
}

// Per-tile id lists in depth order: every Gaussian, taken in depth order, is
// appended to each tile of its rectangle.
std::vector<std::vector<int64_t>> tile_lists(const std::vector<Proj>& pr,
                                             const std::vector<int64_t>& order, int ntx, int nty) {
    std::vector<std::vector<int64_t>> lists((size_t)ntx * nty);
    for (int64_t g : order) {
        const Proj& p = pr[g];
        for (int ty = p.ty0; ty < p.ty1; ++ty)
            for (int tx = p.tx0; tx < p.tx1; ++tx) lists[(size_t)ty * ntx + tx].push_back(g);
    }
    return lists;
}

std::vector<Proj> project_all(const double* P, int64_t n, int64_t ld, int degree, const Cam& cam,
                              int tw, int th) {
    std::vector<Proj> pr((size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) project(P, n, ld, degree, g, cam, tw, th, pr[g]);
    return pr;
}

// One pixel's front-to-back walk over a candidate list (eq. 2).  A candidate
// is a member iff power >= -4.5 (inside its 3-sigma ellipse) and
// alpha = min(0.99, o exp(power)) >= 1/255; the walk stops before the member
// that would take the transmittance below 1e-4.
struct Member { int64_t g; int64_t idx; double alpha, G, T, dx, dy; bool capped; };

struct PixelResult {
    double C[3];
    double T;
    int64_t last;                 // list index + 1 of the last member, 0 if none
    int64_t n_members;
    double m_value, m_grad, ztie;
    uint64_t hash;
    std::vector<Member> members;
};

void walk_pixel(const std::vector<Proj>& pr, const std::vector<int64_t>& list, double px, double py,
                bool keep_members, PixelResult& r) {
    r.C[0] = r.C[1] = r.C[2] = 0;
    r.T = 1.0;
    r.last = 0;
    r.n_members = 0;
    r.m_value = r.m_grad = r.ztie = kInf;
    r.hash = 1469598103934665603ull;
    r.members.clear();
    float prev_z = 0;
    bool have_prev = false;
    for (size_t i = 0; i < list.size(); ++i) {
        const Proj& p = pr[list[i]];
        double dx = p.u - px, dy = p.v - py;
        double power = -0.5 * (p.conic[0] * dx * dx + p.conic[2] * dy * dy) - p.conic[1] * dx * dy;
        r.m_value = std::min(r.m_value, std::fabs(power - kPowerFloor) / -kPowerFloor);
        if (power < kPowerFloor) continue;
        double G = std::exp(power);
        double oG = p.opacity * G;
        double alpha = std::min(kAlphaMax, oG);
        r.m_grad = std::min(r.m_grad, std::fabs(oG - kAlphaMax) / kAlphaMax);
        r.m_value = std::min(r.m_value, std::fabs(alpha - kAlphaMin) / kAlphaMin);
        if (alpha < kAlphaMin) continue;
        if (have_prev) r.ztie = std::min(r.ztie, std::fabs((double)p.z32 - (double)prev_z) / (double)p.z32);
        prev_z = p.z32;
        have_prev = true;
        double Tn = r.T * (1.0 - alpha);
        r.m_value = std::min(r.m_value, std::fabs(Tn - kTMin) / kTMin);
        r.hash = (r.hash ^ (uint64_t)(list[i] * 2 + (oG > kAlphaMax))) * 1099511628211ull;
        if (Tn < kTMin) {
            r.hash = (r.hash ^ 0x9e3779b97f4a7c15ull) * 1099511628211ull;
            break;
        }
        if (keep_members) r.members.push_back({list[i], (int64_t)i, alpha, G, r.T, dx, dy, oG > kAlphaMax});
        for (int ch = 0; ch < 3; ++ch) r.C[ch] += p.rgb[ch] * alpha * r.T;
        r.T = Tn;
        r.last = (int64_t)i + 1;
        r.n_members += 1;
    }
}

// Chain rule from the 2-D quantities (u, v, conic, opacity, rgb) of one view
// to every parameter of the Gaussian; adds into gsum[R] (and, with band
// masks, dL/dM of bands 1..3 into gsum[R .. R + 2]).
void chain_to_params(const Proj& p, const Cam& cam, int degree, const double* P, int64_t ld, int64_t g,
                     const double* d2, double* gsum) {
    auto par = [&](int row) { return P[(int64_t)row * ld + g]; };
    double dmu[3] = {0, 0, 0};
    int K = (degree + 1) * (degree + 1);

    // Colour: rgb = max(0, sum_k f_k B_k(dir) + 0.5).
    double draw[3];
    for (int ch = 0; ch < 3; ++ch) draw[ch] = p.clamped[ch] ? 0.0 : d2[6 + ch];
    double B[16], dB[16][3];
    sh_basis(degree, p.dn[0], p.dn[1], p.dn[2], B, dB);
    // With band masks the coefficient is M_l f; gsum[R + l - 1] collects
    // dL/dM_l = sum over band l's coefficients of dL/d(M_l f) f.
    const int R = 11 + 3 * K;
    double ddn[3] = {0, 0, 0};
    for (int k = 0; k < K; ++k) {
        const int l = sh_band(k);
        const double M = band_gate(g, l);
        for (int ch = 0; ch < 3; ++ch) {
            const double f = par(11 + 3 * k + ch);
            gsum[11 + 3 * k + ch] += M * draw[ch] * B[k];
            if (g_shm && l > 0) gsum[R + l - 1] += draw[ch] * B[k] * f;
            for (int a = 0; a < 3; ++a) ddn[a] += draw[ch] * M * f * dB[k][a];
        }
    }
    double dot = ddn[0] * p.dn[0] + ddn[1] * p.dn[1] + ddn[2] * p.dn[2];
    for (int a = 0; a < 3; ++a) dmu[a] += (ddn[a] - p.dn[a] * dot) / p.dlen;

    // Opacity: o = sigmoid(logit), do/dlogit = o (1 - o); or o = |x|,
    // do/dx = sign(x) (0 at x = 0).
    if (g_opacity_act) {
        const double x = par(10);
        gsum[10] += x > 0 ? d2[5] : (x < 0 ? -d2[5] : 0.0);
    } else {
        gsum[10] += d2[5] * p.opacity * (1.0 - p.opacity);
    }

    // Conic K = A^-1 with A = [[a, b], [b, c]] (dilated).  Matrix gradient of
    // the symmetric K: GK = [[dL/dca, dL/dcb / 2], [dL/dcb / 2, dL/dcc]];
    // dK = -K dA K gives GA = -K GK K.
    double Km[2][2] = {{p.conic[0], p.conic[1]}, {p.conic[1], p.conic[2]}};
    double GK[2][2] = {{d2[2], 0.5 * d2[3]}, {0.5 * d2[3], d2[4]}};
    double KG[2][2], GA[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) KG[i][j] = Km[i][0] * GK[0][j] + Km[i][1] * GK[1][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) GA[i][j] = -(KG[i][0] * Km[0][j] + KG[i][1] * Km[1][j]);

    // A = T Sigma T^T (+ dilation): dL/dSigma = T^T GA T, dL/dT = 2 GA T Sigma.
    double GS[3][3], GT[2][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += p.T[k][i] * GA[k][l] * p.T[l][j];
            GS[i][j] = acc;
        }
    double TS[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += p.T[i][k] * p.Sigma[k][j];
            TS[i][j] = acc;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) GT[i][j] = 2.0 * (GA[i][0] * TS[0][j] + GA[i][1] * TS[1][j]);
    // T = J W: dL/dJ = dL/dT W^T.
    double GJ[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += GT[i][k] * cam.R[j][k];
            GJ[i][j] = acc;
        }
    // J = [[fx/z, 0, -fx rx/z], [0, fy/z, -fy ry/z]] where rx is x/z unless the
    // tangent clamp held it at a constant.
    double x = p.xc[0], y = p.xc[1], z = p.z;
    double dxc[3] = {0, 0, 0};
    dxc[2] += GJ[0][0] * (-cam.fx / (z * z)) + GJ[1][1] * (-cam.fy / (z * z));
    if (!p.clx) {
        dxc[0] += GJ[0][2] * (-cam.fx / (z * z));
        dxc[2] += GJ[0][2] * (2.0 * cam.fx * x / (z * z * z));
    } else {
        dxc[2] += GJ[0][2] * (cam.fx * p.rxc / (z * z));
    }
    if (!p.cly) {
        dxc[1] += GJ[1][2] * (-cam.fy / (z * z));
        dxc[2] += GJ[1][2] * (2.0 * cam.fy * y / (z * z * z));
    } else {
        dxc[2] += GJ[1][2] * (cam.fy * p.ryc / (z * z));
    }
    // Screen mean: u = fx x / z + cx, v = fy y / z + cy.
    dxc[0] += d2[0] * cam.fx / z;
    dxc[2] += -d2[0] * cam.fx * x / (z * z);
    dxc[1] += d2[1] * cam.fy / z;
    dxc[2] += -d2[1] * cam.fy * y / (z * z);
    // Camera transform xc = W mu + t.
    for (int a = 0; a < 3; ++a) dmu[a] += cam.R[0][a] * dxc[0] + cam.R[1][a] * dxc[1] + cam.R[2][a] * dxc[2];
    for (int a = 0; a < 3; ++a) gsum[a] += dmu[a];

    // Sigma = M M^T with M = R S: dL/dM = 2 dL/dSigma M.
    double GM[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += GS[i][k] * p.M[k][j];
            GM[i][j] = 2.0 * acc;
        }
    double GR[3][3];
    for (int j = 0; j < 3; ++j) {
        double ds = 0;
        for (int i = 0; i < 3; ++i) {
            ds += GM[i][j] * p.Rq[i][j];
            GR[i][j] = GM[i][j] * p.s[j];
        }
        gsum[3 + j] += ds * p.s[j];                            // d/d log-scale
    }
    // R(q) for the unit quaternion (w, x, y, z).
    double w = p.qn[0], qx = p.qn[1], qy = p.qn[2], qz = p.qn[3];
    double dq[4];
    dq[0] = 2 * (-qz * GR[0][1] + qy * GR[0][2] + qz * GR[1][0] - qx * GR[1][2] - qy * GR[2][0] + qx * GR[2][1]);
    dq[1] = 2 * (qy * GR[0][1] + qz * GR[0][2] + qy * GR[1][0] - 2 * qx * GR[1][1] - w * GR[1][2]
                 + qz * GR[2][0] + w * GR[2][1] - 2 * qx * GR[2][2]);
    dq[2] = 2 * (-2 * qy * GR[0][0] + qx * GR[0][1] + w * GR[0][2] + qx * GR[1][0] + qz * GR[1][2]
                 - w * GR[2][0] + qz * GR[2][1] - 2 * qy * GR[2][2]);
    dq[3] = 2 * (-2 * qz * GR[0][0] - w * GR[0][1] + qx * GR[0][2] + w * GR[1][0] - 2 * qz * GR[1][1]
                 + qy * GR[1][2] + qx * GR[2][0] + qy * GR[2][1]);
    // Normalisation q_hat = q / |q|.
    double qd = w * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
    for (int i = 0; i < 4; ++i) gsum[6 + i] += (dq[i] - p.qn[i] * qd) / p.qnorm;
}

}  // namespace

extern "C" {

// Threads the OpenMP loops of the oracle use.
int oracle_num_threads() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// Selects the opacity activation of later calls (0 sigmoid, 1 absolute value).
void oracle_set_opacity_activation(int act) { g_opacity_act = act ? 1 : 0; }

// SH-band masks of later calls: logits [3][ld] (nullptr: off), the gate
// threshold on sigmoid(logit), and where the backward writes dL/dlogit
// ([3][ld], or nullptr).  The arrays must outlive the calls that use them.
void oracle_set_sh_mask(const double* logits, int64_t ld, double threshold, double* grad_out) {
    g_shm = logits;
    g_shm_ld = ld;
    g_shm_threshold = threshold;
    g_shm_grad = grad_out;
}

// Sets the threads of later OpenMP loops (timing at 1 thread and at all cores).
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

// Number of doubles per projected record written by oracle_project.
int oracle_nrec() { return 40; }

// Record layout: 0 visible, 1 u, 2 v, 3 z, 4 float32(z), 5 a, 6 b, 7 c,
// 8 det, 9..11 conic, 12 ex, 13 ey, 14 tx0, 15 tx1, 16 ty0, 17 ty1 (tile
// rect, exclusive ends), 18..20 rgb, 21..23 colour-clamp flags, 24 opacity,
// 25 near margin, 26 det margin, 27 rect margin (px), 28 tangent margin,
// 29 colour margin, 30/31 tangent clamp flags, 32..34 camera-space mean.
int oracle_project(const double* params, int64_t n, int64_t ld, int32_t degree, const double* camv,
                   int32_t tile_w, int32_t tile_h, double* rec) {
    Cam cam = read_cam(camv);
    std::vector<Proj> pr = project_all(params, n, ld, degree, cam, tile_w, tile_h);
    for (int64_t g = 0; g < n; ++g) {
        const Proj& p = pr[g];
        double* r = rec + g * 40;
        for (int i = 0; i < 40; ++i) r[i] = 0;
        r[0] = p.visible; r[1] = p.u; r[2] = p.v; r[3] = p.z; r[4] = (double)p.z32;
        r[5] = p.a; r[6] = p.b; r[7] = p.c; r[8] = p.det;
        r[9] = p.conic[0]; r[10] = p.conic[1]; r[11] = p.conic[2];
        r[12] = p.ex; r[13] = p.ey;
        r[14] = p.tx0; r[15] = p.tx1; r[16] = p.ty0; r[17] = p.ty1;
        for (int ch = 0; ch < 3; ++ch) { r[18 + ch] = p.rgb[ch]; r[21 + ch] = p.clamped[ch]; }
        r[24] = p.opacity;
        r[25] = p.m_near; r[26] = p.m_det; r[27] = p.m_rect; r[28] = p.m_tan; r[29] = p.m_col;
        r[30] = p.clx; r[31] = p.cly;
        for (int i = 0; i < 3; ++i) r[32 + i] = p.xc[i];
    }
    return 0;
}

// Tile binning: per-tile counts [ntx*nty] and, if ids != NULL, the
// concatenated per-tile id lists (tile-major, depth order within a tile).
// Returns the total number of (tile, Gaussian) instances.
int64_t oracle_bin(const double* params, int64_t n, int64_t ld, int32_t degree, const double* camv,
                   int32_t tile_w, int32_t tile_h, int64_t* counts, int64_t* ids, int64_t* order_out,
                   int64_t* n_visible) {
    Cam cam = read_cam(camv);
    std::vector<Proj> pr = project_all(params, n, ld, degree, cam, tile_w, tile_h);
    std::vector<int64_t> order = depth_order(pr);
    int ntx = (cam.W + tile_w - 1) / tile_w, nty = (cam.H + tile_h - 1) / tile_h;
    auto lists = tile_lists(pr, order, ntx, nty);
    int64_t total = 0;
    for (size_t t = 0; t < lists.size(); ++t) {
        if (counts) counts[t] = (int64_t)lists[t].size();
        if (ids) std::memcpy(ids + total, lists[t].data(), lists[t].size() * sizeof(int64_t));
        total += (int64_t)lists[t].size();
    }
    if (order_out) std::memcpy(order_out, order.data(), order.size() * sizeof(int64_t));
    if (n_visible) *n_visible = (int64_t)order.size();
    return total;
}

// Forward render of one view (eq. 2).  brute != 0 walks every visible
// Gaussian in depth order for every pixel instead of the pixel's tile list.
// Outputs: image [3][H][W] (colour + T_final * bg), T_final [H][W], last
// [H][W] (tile-list index + 1 of the last member), n_members [H][W],
// m_value / m_grad / ztie [H][W] (smallest relative distance of any decision
// from its threshold; nearest depth gap between consecutive members) and a
// per-pixel hash of the member set.
int oracle_render(const double* params, int64_t n, int64_t ld, int32_t degree, const double* camv,
                  int32_t tile_w, int32_t tile_h, const double* bg, int32_t brute, double* image,
                  double* T_final, int64_t* last, int64_t* n_members, double* m_value, double* m_grad,
                  double* ztie, uint64_t* hash) {
    Cam cam = read_cam(camv);
    std::vector<Proj> pr = project_all(params, n, ld, degree, cam, tile_w, tile_h);
    std::vector<int64_t> order = depth_order(pr);
    int ntx = (cam.W + tile_w - 1) / tile_w, nty = (cam.H + tile_h - 1) / tile_h;
    std::vector<std::vector<int64_t>> lists;
    if (!brute) lists = tile_lists(pr, order, ntx, nty);
    const int64_t HW = (int64_t)cam.W * cam.H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int py = 0; py < cam.H; ++py) {
        PixelResult r;
        for (int px = 0; px < cam.W; ++px) {
            const std::vector<int64_t>& list =
                brute ? order : lists[(size_t)(py / tile_h) * ntx + (px / tile_w)];
            walk_pixel(pr, list, (double)px, (double)py, false, r);
            int64_t o = (int64_t)py * cam.W + px;
            for (int ch = 0; ch < 3; ++ch) image[ch * HW + o] = r.C[ch] + r.T * bg[ch];
            if (T_final) T_final[o] = r.T;
            if (last) last[o] = r.last;
            if (n_members) n_members[o] = r.n_members;
            if (m_value) m_value[o] = r.m_value;
            if (m_grad) m_grad[o] = r.m_grad;
            if (ztie) ztie[o] = r.ztie;
            if (hash) hash[o] = r.hash;
        }
    }
    return 0;
}

// Sampled pixels of one view by the brute-force walk over every visible
// Gaussian in depth order (the compositing of eq. 2 without tiles; equal to
// the tiled render).  pix [m][2] = (px, py); out [m][3] colour (+ T_final*bg),
// T_final [m], m_value [m] (smallest relative distance of a decision from
// its threshold).
int oracle_render_pixels(const double* params, int64_t n, int64_t ld, int32_t degree, const double* camv,
                         const double* bg, const int64_t* pix, int64_t m, double* out, double* T_final,
                         double* m_value) {
    Cam cam = read_cam(camv);
    std::vector<Proj> pr = project_all(params, n, ld, degree, cam, 16, 16);
    std::vector<int64_t> order = depth_order(pr);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        PixelResult r;
        walk_pixel(pr, order, (double)pix[2 * i], (double)pix[2 * i + 1], false, r);
        for (int ch = 0; ch < 3; ++ch) out[3 * i + ch] = r.C[ch] + r.T * bg[ch];
        T_final[i] = r.T;
        m_value[i] = r.m_value;
    }
    return 0;
}

// Backward of the render (Section 3.2.4) for n_views views that share one
// parameter block; the gradient of every parameter is summed over the views.
// dL_dimage is [V][3][H][W].  Rows of frozen Gaussians (frozen[g] != 0) are
// left untouched in grads [R][ld]; active rows are overwritten.  Optional
// outputs: grad2d [V][9][n] (dL/d(u, v, conic_a, conic_b, conic_c, opacity,
// r, g, b)) and visible [V][n].
//
// Per pixel with members i = 1..m (alpha_i, T_i, colour c_i):
//   dC/dc_i     = alpha_i T_i
//   dC/dalpha_i = c_i T_i - (sum_{j>i} c_j alpha_j T_j + T_final bg) / (1 - alpha_i)
// computed with explicit suffix sums.
int oracle_render_backward(const double* params, int64_t n, int64_t ld, int32_t degree,
                           const double* cams, int32_t n_views, int32_t tile_w, int32_t tile_h,
                           const double* bg, const double* dL_dimage, const uint8_t* frozen,
                           double* grads, double* grad2d, uint8_t* visible_out) {
    const int R = 11 + 3 * (degree + 1) * (degree + 1);
    const int RX = R + 3;    // + the three band-mask gradients dL/dM_l
    std::vector<double> total((size_t)RX * n, 0.0);
    std::vector<uint8_t> any_visible((size_t)n, 0);
    int64_t img_off = 0;
    for (int v = 0; v < n_views; ++v) {
        Cam cam = read_cam(cams + 22 * v);
        std::vector<Proj> pr = project_all(params, n, ld, degree, cam, tile_w, tile_h);
        std::vector<int64_t> order = depth_order(pr);
        int ntx = (cam.W + tile_w - 1) / tile_w, nty = (cam.H + tile_h - 1) / tile_h;
        auto lists = tile_lists(pr, order, ntx, nty);
        const int64_t HW = (int64_t)cam.W * cam.H;
        const double* dLv = dL_dimage + img_off;
        img_off += 3 * HW;

        int nthreads = 1;
#ifdef _OPENMP
        nthreads = omp_get_max_threads();
#endif
        std::vector<double> part((size_t)nthreads * 9 * n, 0.0);
#pragma omp parallel num_threads(nthreads)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* acc = part.data() + (size_t)tid * 9 * n;
            PixelResult r;
            std::vector<double> suffix;
            // static schedule: the rows each thread sums are fixed, so the
            // result does not depend on timing
#pragma omp for schedule(static)
            for (int py = 0; py < cam.H; ++py) {
                for (int px = 0; px < cam.W; ++px) {
                    const auto& list = lists[(size_t)(py / tile_h) * ntx + (px / tile_w)];
                    walk_pixel(pr, list, (double)px, (double)py, true, r);
                    int64_t o = (int64_t)py * cam.W + px;
                    double dC[3] = {dLv[o], dLv[HW + o], dLv[2 * HW + o]};
                    size_t m = r.members.size();
                    // suffix[i] = sum_{j > i} c_j alpha_j T_j (per channel)
                    suffix.assign(3 * (m + 1), 0.0);
                    for (size_t k = m; k-- > 0;) {
                        const Member& e = r.members[k];
                        const Proj& p = pr[e.g];
                        for (int ch = 0; ch < 3; ++ch)
                            suffix[3 * k + ch] = suffix[3 * (k + 1) + ch] + p.rgb[ch] * e.alpha * e.T;
                    }
                    for (size_t k = 0; k < m; ++k) {
                        const Member& e = r.members[k];
                        const Proj& p = pr[e.g];
                        double dalpha = 0;
                        for (int ch = 0; ch < 3; ++ch) {
                            acc[(6 + ch) * n + e.g] += dC[ch] * e.alpha * e.T;
                            double behind = suffix[3 * (k + 1) + ch] + r.T * bg[ch];
                            dalpha += dC[ch] * (p.rgb[ch] * e.T - behind / (1.0 - e.alpha));
                        }
                        if (e.capped) continue;                 // alpha held at 0.99
                        // alpha = o * exp(power);  power = -0.5 d^T K d, d = (u - px, v - py)
                        double dpower = dalpha * e.alpha;
                        acc[5 * n + e.g] += dalpha * e.G;
                        acc[0 * n + e.g] += dpower * -(p.conic[0] * e.dx + p.conic[1] * e.dy);
                        acc[1 * n + e.g] += dpower * -(p.conic[1] * e.dx + p.conic[2] * e.dy);
                        acc[2 * n + e.g] += dpower * -0.5 * e.dx * e.dx;
                        acc[3 * n + e.g] += dpower * -e.dx * e.dy;
                        acc[4 * n + e.g] += dpower * -0.5 * e.dy * e.dy;
                    }
                }
            }
        }
        std::vector<double> d2((size_t)9 * n, 0.0);
        for (int t = 0; t < nthreads; ++t)
            for (size_t i = 0; i < (size_t)9 * n; ++i) d2[i] += part[(size_t)t * 9 * n + i];
        if (grad2d)
            for (size_t i = 0; i < (size_t)9 * n; ++i) grad2d[(size_t)v * 9 * n + i] = d2[i];
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            if (visible_out) visible_out[(size_t)v * n + g] = pr[g].visible;
            if (!pr[g].visible) continue;
            any_visible[g] = 1;
            if (frozen && frozen[g]) continue;
            double d[9], gs[64];
            for (int k = 0; k < 9; ++k) d[k] = d2[(size_t)k * n + g];
            for (int k = 0; k < RX; ++k) gs[k] = 0;
            chain_to_params(pr[g], cam, degree, params, ld, g, d, gs);
            for (int k = 0; k < RX; ++k) total[(size_t)k * n + g] += gs[k];
        }
    }
    for (int64_t g = 0; g < n; ++g) {
        if (frozen && frozen[g]) continue;
        for (int k = 0; k < R; ++k) grads[(size_t)k * ld + g] = total[(size_t)k * n + g];
        if (g_shm && g_shm_grad)
            for (int l = 1; l <= 3; ++l) {   // straight-through: dL/dlogit = dL/dM sigmoid'(logit)
                const double sg = sigmoid(g_shm[(int64_t)(l - 1) * g_shm_ld + g]);
                g_shm_grad[(int64_t)(l - 1) * g_shm_ld + g] = total[(size_t)(R + l - 1) * n + g] * sg * (1.0 - sg);
            }
    }
    return 0;
}

// Real SH basis at unit directions, for quadrature and symmetry checks:
// dirs [m][3] -> out [m][(degree+1)^2] (and grad [m][K][3] if not NULL).
int oracle_sh_basis(int32_t degree, const double* dirs, int64_t m, double* out, double* grad) {
    int K = (degree + 1) * (degree + 1);
    for (int64_t i = 0; i < m; ++i) {
        double B[16], dB[16][3];
        sh_basis(degree, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], B, dB);
        for (int k = 0; k < K; ++k) {
            out[i * K + k] = B[k];
            if (grad)
                for (int a = 0; a < 3; ++a) grad[(i * K + k) * 3 + a] = dB[k][a];
        }
    }
    return 0;
}

}  // extern "C"
