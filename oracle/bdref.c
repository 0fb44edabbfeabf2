/*
 * bdref.c -- plain CPU oracle (TEST INFRASTRUCTURE ONLY; see bdref.h).
 *
 * Each function writes out the definition it follows as directly as
 * possible.  Floating point is FP64 throughout and is compiled without
 * contraction (-ffp-contract=off), so every rounding step is a plain IEEE
 * operation in the order written here.
 *
 * Readings where the paper is silent (pixel grid, rounding of box centres,
 * image-border policy, histogram layout) are stated at each function.
 */
#include "bdref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ integral image */

/* Sec. III-A: box averages come from an integral image.  Reading: the integral
 * image has a zero first row and column, and entry (y+1, x+1) is the sum of
 * all pixels above and to the left of (y, x) inclusive.  Built row by row with
 * the four-term recurrence, in u32 arithmetic (modulo 2^32). */
void bdref_build_integral(const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch,
                          uint32_t* ii, int64_t ii_pitch)
{
    for (int32_t x = 0; x <= W; ++x) ii[x] = 0u;
    for (int32_t y = 0; y < H; ++y) {
        uint32_t* above = ii + (int64_t)y * ii_pitch;
        uint32_t* row = ii + (int64_t)(y + 1) * ii_pitch;
        row[0] = 0u;
        for (int32_t x = 0; x < W; ++x) {
            uint32_t pixel = img[(int64_t)y * img_pitch + x];
            row[x + 1] = pixel + above[x + 1] + row[x] - above[x];
        }
    }
}

/* ------------------------------------------------------------------ keypoints */

int32_t bdref_keypoint_valid(const bdref_keypoint* kp)
{
    return isfinite(kp->x) && isfinite(kp->y) && isfinite(kp->scale) && isfinite(kp->angle) &&
           kp->scale > 0.0f;
}

/* Reading of the patch frame (the paper only says boxes are centred at pixels
 * u of the normalized patch): a normalized-patch offset u = (ux, uy) maps to
 * the image point p = c + scale * R(angle) u, with R the rotation taking the
 * patch x axis to (cos a, sin a).  Evaluated in FP64 in exactly this order. */
static void patch_to_image(double cx, double cy, double sa, double sb, double ux, double uy,
                           double* px, double* py)
{
    /* sa = scale*cos(angle), sb = scale*sin(angle) */
    *px = cx + (sa * ux - sb * uy);
    *py = cy + (sb * ux + sa * uy);
}

/* ------------------------------------------------------------------ BAD */

/* Sum of the (2R+1)^2 pixels centred at (cx, cy), from four integral-image
 * corners.  The true sum is below 2^32, so u32 wrap-around cancels. */
static int64_t box_sum(const uint32_t* ii, int64_t pitch, int64_t cx, int64_t cy, int64_t R)
{
    uint32_t top_left = ii[(cy - R) * pitch + (cx - R)];
    uint32_t top_right = ii[(cy - R) * pitch + (cx + R + 1)];
    uint32_t bottom_left = ii[(cy + R + 1) * pitch + (cx - R)];
    uint32_t bottom_right = ii[(cy + R + 1) * pitch + (cx + R + 1)];
    uint32_t s = bottom_right - top_right - bottom_left + top_left;
    return (int64_t)s;
}

/* distance of v to the nearest integer, for the near-tie audit */
static double dist_to_integer(double v) { return fabs(v - floor(v + 0.5)); }

/* Box centre from a patch point: round half up to the pixel grid, then
 * clamp so that the whole box of radius R lies inside [0, n). */
static int64_t box_centre(double p, int64_t R, int64_t n, int64_t* near_ties)
{
    double q = p + 0.5;
    double d = dist_to_integer(q);
    if (d > 0.0 && d < 1e-9) ++*near_ties;
    double c = floor(q);
    if (c < (double)R) c = (double)R;
    if (c > (double)(n - 1 - R)) c = (double)(n - 1 - R);
    return (int64_t)c;
}

/* Sec. III-A.  Weak descriptor h(x; f, theta) = +1 if f(x) <= theta else -1,
 * where f(x; u1, u2, s) = mean grey level of the box of side s at u1 minus the
 * mean of the box of side s at u2.  The bit stored is 1 for h = +1.
 *
 * Readings: the box radius in image pixels is R = floor(r*scale + 0.5),
 * capped so a box fits the image; both boxes share it (side s = 2R+1).  The
 * box centres are the patch points rounded half up and clamped so the box
 * stays inside the image.  With area A = s^2, f <= theta is evaluated exactly
 * as S1 - S2 <= theta * A (S = box sums; theta*A is exact in FP64).
 * Keypoints with non-finite fields or scale <= 0 get an all-zero code. */
int64_t bdref_describe_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch,
                           const bdref_keypoint* kps, int32_t n_kp,
                           const bdref_box_pair* pairs, int32_t n_bits, uint64_t* codes)
{
    const int32_t n_words = n_bits / 64;
    const int64_t r_cap = ((W < H ? W : H) - 1) / 2;
    int64_t near_ties = 0;
    for (int32_t i = 0; i < n_kp; ++i) {
        uint64_t* code = codes + (int64_t)i * n_words;
        memset(code, 0, sizeof(uint64_t) * (size_t)n_words);
        const bdref_keypoint* kp = &kps[i];
        if (!bdref_keypoint_valid(kp)) continue;
        double scale = (double)kp->scale;
        double angle = (double)kp->angle;
        double sa = scale * cos(angle);
        double sb = scale * sin(angle);
        for (int32_t j = 0; j < n_bits; ++j) {
            const bdref_box_pair* pr = &pairs[j];
            double rr = floor((double)pr->radius * scale + 0.5);
            int64_t R = rr > (double)r_cap ? r_cap : (int64_t)rr;
            double p1x, p1y, p2x, p2y;
            patch_to_image(kp->x, kp->y, sa, sb, pr->x1, pr->y1, &p1x, &p1y);
            patch_to_image(kp->x, kp->y, sa, sb, pr->x2, pr->y2, &p2x, &p2y);
            int64_t c1x = box_centre(p1x, R, W, &near_ties);
            int64_t c1y = box_centre(p1y, R, H, &near_ties);
            int64_t c2x = box_centre(p2x, R, W, &near_ties);
            int64_t c2y = box_centre(p2y, R, H, &near_ties);
            int64_t s1 = box_sum(ii, ii_pitch, c1x, c1y, R);
            int64_t s2 = box_sum(ii, ii_pitch, c2x, c2y, R);
            int64_t side = 2 * R + 1;
            double area = (double)(side * side);
            int bit = (double)(s1 - s2) <= (double)pr->threshold * area;
            if (bit) code[j / 64] |= (uint64_t)1 << (j % 64);
        }
    }
    return near_ties;
}

/* ------------------------------------------------------------------ HashSIFT */

static double pixel_value(const void* img, int32_t dtype, int64_t pitch, int64_t x, int64_t y)
{
    const unsigned char* row = (const unsigned char*)img + y * pitch;
    if (dtype == 0) return (double)row[x] / 255.0;
    float v;
    memcpy(&v, row + 4 * x, sizeof v);
    return (double)v;
}

static int64_t clamp_index(double v, int64_t n)
{
    if (v < 0.0) return 0;
    if (v > (double)(n - 1)) return n - 1;
    return (int64_t)v;
}

/* Bilinear interpolation at (px, py) with clamp-to-edge addressing, written
 * as nested linear interpolation a + t (b - a): the same polynomial as the
 * weighted four-tap form, but exact wherever the four pixels are equal, so a
 * flat image region gives exactly zero gradients. */
static double bilinear(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t pitch,
                       double px, double py)
{
    double x0 = floor(px), y0 = floor(py);
    double fx = px - x0, fy = py - y0;
    int64_t xa = clamp_index(x0, W), xb = clamp_index(x0 + 1.0, W);
    int64_t ya = clamp_index(y0, H), yb = clamp_index(y0 + 1.0, H);
    double v00 = pixel_value(img, dtype, pitch, xa, ya);
    double v01 = pixel_value(img, dtype, pitch, xb, ya);
    double v10 = pixel_value(img, dtype, pitch, xa, yb);
    double v11 = pixel_value(img, dtype, pitch, xb, yb);
    double top = v00 + fx * (v01 - v00);
    double bottom = v10 + fx * (v11 - v10);
    return top + fy * (bottom - top);
}

#define PATCH 32
#define APRON 34 /* 32x32 patch plus a one-pixel apron for central differences */

/* Sec. III-B takes the SIFT feature vector of the normalized 32x32 patch
 * (the timing experiment describes only that patch, with no image pyramid).
 * The paper fixes no further detail; the reading here is Lowe's descriptor
 * layout on that patch:
 *   1. patch pixel (i, j), i, j in -1..32, is the bilinear sample at patch
 *      offset u = (j - 15.5, i - 15.5), clamp-to-edge;
 *   2. central differences gx = P[i][j+1] - P[i][j-1], gy = P[i+1][j] - P[i-1][j];
 *      magnitude m and angle phi = atan2(gy, gx) in [0, 2 pi) (the patch is
 *      sampled in the rotated frame, so phi is relative to the keypoint angle);
 *   3. weight m * exp(-((j-15.5)^2 + (i-15.5)^2) / (2 * 16^2));
 *   4. trilinear vote into 4x4 spatial cells (cell centres at 8c + 3.5) and 8
 *      orientation bins (bin centres at 2 pi o / 8, circular); cells outside
 *      0..3 are dropped; index (cy * 4 + cx) * 8 + o;
 *   5. L2 normalization (a zero histogram stays zero); no clipping.
 * Keypoints with non-finite fields or scale <= 0 give a zero histogram. */
void bdref_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                         const bdref_keypoint* kps, int32_t n_kp, double* hist)
{
    const double two_pi = 2.0 * M_PI;
    double patch[APRON][APRON];
    for (int32_t n = 0; n < n_kp; ++n) {
        double* h = hist + (int64_t)n * 128;
        for (int b = 0; b < 128; ++b) h[b] = 0.0;
        const bdref_keypoint* kp = &kps[n];
        if (!bdref_keypoint_valid(kp)) continue;
        double scale = (double)kp->scale;
        double sa = scale * cos((double)kp->angle);
        double sb = scale * sin((double)kp->angle);

        for (int i = -1; i <= PATCH; ++i)
            for (int j = -1; j <= PATCH; ++j) {
                double px, py;
                patch_to_image(kp->x, kp->y, sa, sb, j - 15.5, i - 15.5, &px, &py);
                patch[i + 1][j + 1] = bilinear(img, dtype, W, H, img_pitch, px, py);
            }

        for (int i = 0; i < PATCH; ++i)
            for (int j = 0; j < PATCH; ++j) {
                double gx = patch[i + 1][j + 2] - patch[i + 1][j];
                double gy = patch[i + 2][j + 1] - patch[i][j + 1];
                double m = sqrt(gx * gx + gy * gy);
                double phi = atan2(gy, gx);
                if (phi < 0.0) phi += two_pi;
                double du = j - 15.5, dv = i - 15.5;
                double w = m * exp(-(du * du + dv * dv) / (2.0 * 16.0 * 16.0));

                double bx = (j + 0.5) / 8.0 - 0.5;
                double by = (i + 0.5) / 8.0 - 0.5;
                double bo = phi * 8.0 / two_pi;
                double x0 = floor(bx), y0 = floor(by), o0 = floor(bo);
                double dx = bx - x0, dy = by - y0, dor = bo - o0;
                for (int ky = 0; ky < 2; ++ky) {
                    int cy = (int)y0 + ky;
                    if (cy < 0 || cy > 3) continue;
                    double wy = ky ? dy : 1.0 - dy;
                    for (int kx = 0; kx < 2; ++kx) {
                        int cx = (int)x0 + kx;
                        if (cx < 0 || cx > 3) continue;
                        double wx = kx ? dx : 1.0 - dx;
                        for (int ko = 0; ko < 2; ++ko) {
                            int o = ((int)o0 + ko) % 8;
                            double wo = ko ? dor : 1.0 - dor;
                            h[(cy * 4 + cx) * 8 + o] += w * wy * wx * wo;
                        }
                    }
                }
            }

        double ss = 0.0;
        for (int b = 0; b < 128; ++b) ss += h[b] * h[b];
        if (ss > 0.0) {
            double norm = sqrt(ss);
            for (int b = 0; b < 128; ++b) h[b] /= norm;
        }
    }
}

/* Sec. III-B: D(x) = sgn(B [f(x); 1]).  Reading: the last column of the
 * paper's B is stored as -t, so the response is r = B f - t, and the bit is
 * 1 when r > 0 (sgn(0) maps to 0). */
void bdref_hashsift_project(const double* hist, int32_t n_kp, const float* B, const float* t,
                            int32_t n_bits, const uint8_t* valid, double* resp, uint64_t* codes)
{
    const int32_t n_words = n_bits / 64;
    for (int32_t n = 0; n < n_kp; ++n) {
        const double* f = hist + (int64_t)n * 128;
        uint64_t* code = codes + (int64_t)n * n_words;
        memset(code, 0, sizeof(uint64_t) * (size_t)n_words);
        for (int32_t j = 0; j < n_bits; ++j) {
            double r = 0.0;
            for (int k = 0; k < 128; ++k) r += (double)B[(int64_t)j * 128 + k] * f[k];
            r -= (double)t[j];
            if (resp) resp[(int64_t)n * n_bits + j] = r;
            if ((valid == NULL || valid[n]) && r > 0.0) code[j / 64] |= (uint64_t)1 << (j % 64);
        }
    }
}

/* ------------------------------------------------------------------ Hamming k-NN */

static uint32_t popcount64(uint64_t v)
{
    uint32_t c = 0;
    while (v) {
        v &= v - 1;
        ++c;
    }
    return c;
}

/* Sec. III-A: S(x, y) = h(x)^T h(y) = K - 2 d_H(x, y), so the most similar
 * train code is the one at the smallest Hamming distance.  Reading: ties in
 * distance go to the lower train index (lexicographic (d, index) order). */
void bdref_match_knn(const uint64_t* query, int32_t n_q, const uint64_t* train, int32_t n_t,
                     int32_t n_words, int32_t k, int32_t* idx, uint32_t* dist)
{
    for (int32_t i = 0; i < n_q; ++i) {
        int32_t* bi = idx + (int64_t)i * k;
        uint32_t* bd = dist + (int64_t)i * k;
        for (int32_t s = 0; s < k; ++s) {
            bi[s] = -1;
            bd[s] = 0xFFFFFFFFu;
        }
        const uint64_t* q = query + (int64_t)i * n_words;
        for (int32_t j = 0; j < n_t; ++j) {
            const uint64_t* tr = train + (int64_t)j * n_words;
            uint32_t d = 0;
            for (int32_t w = 0; w < n_words; ++w) d += popcount64(q[w] ^ tr[w]);
            /* j increases, so an equal distance never displaces an earlier index */
            if (bi[k - 1] >= 0 && d >= bd[k - 1]) continue;
            int32_t s = k - 1;
            while (s > 0 && (bi[s - 1] < 0 || d < bd[s - 1])) {
                bi[s] = bi[s - 1];
                bd[s] = bd[s - 1];
                --s;
            }
            bi[s] = j;
            bd[s] = d;
        }
    }
}

static uint32_t hamming(const uint64_t* a, const uint64_t* b, int32_t n_words)
{
    uint32_t d = 0;
    for (int32_t w = 0; w < n_words; ++w) d += popcount64(a[w] ^ b[w]);
    return d;
}

int32_t bdref_match_mutual(const uint64_t* query, int32_t n_q, const uint64_t* train, int32_t n_t,
                           int32_t n_words, double max_ratio, int32_t* match, uint32_t* dist, double* ratio)
{
    int32_t count = 0;
    for (int32_t i = 0; i < n_q; ++i) {
        const uint64_t* q = query + (int64_t)i * n_words;
        /* nearest train code of query i, then the smallest distance among the others */
        int32_t j1 = -1;
        uint32_t d1 = 0xFFFFFFFFu;
        for (int32_t j = 0; j < n_t; ++j) {
            const uint32_t d = hamming(q, train + (int64_t)j * n_words, n_words);
            if (j1 < 0 || d < d1) {
                j1 = j;
                d1 = d;
            }
        }
        int have_d2 = 0;
        uint32_t d2 = 0xFFFFFFFFu;
        for (int32_t j = 0; j < n_t; ++j) {
            if (j == j1) continue;
            const uint32_t d = hamming(q, train + (int64_t)j * n_words, n_words);
            if (!have_d2 || d < d2) {
                have_d2 = 1;
                d2 = d;
            }
        }
        dist[i] = d1;
        if (ratio) ratio[i] = !have_d2 ? 0.0 : (d2 == 0 ? 1.0 : (double)d1 / (double)d2);
        match[i] = -1;
        if (j1 < 0) continue;
        /* nearest query of train j1 */
        const uint64_t* t = train + (int64_t)j1 * n_words;
        int32_t back = -1;
        uint32_t db = 0xFFFFFFFFu;
        for (int32_t r = 0; r < n_q; ++r) {
            const uint32_t d = hamming(t, query + (int64_t)r * n_words, n_words);
            if (back < 0 || d < db) {
                back = r;
                db = d;
            }
        }
        if (back != i) continue;
        if (max_ratio > 0.0 && have_d2 && !((double)d1 < max_ratio * (double)d2)) continue;
        match[i] = j1;
        ++count;
    }
    return count;
}

/* ------------------------------------------------------------------ reduced precision */

float bdref_round_bf16(float x)
{
    uint32_t bits;
    memcpy(&bits, &x, sizeof bits);
    if ((bits & 0x7f800000u) == 0x7f800000u) return x; /* inf / nan unchanged */
    uint32_t lsb = (bits >> 16) & 1u;
    bits += 0x7fffu + lsb; /* round to nearest, ties to even */
    bits &= 0xffff0000u;
    float y;
    memcpy(&y, &bits, sizeof y);
    return y;
}

/* e4m3: normal numbers 2^e * (1 + m/8) for e in [-6, 8] (m <= 6 at e = 8),
 * subnormals k * 2^-9.  The quantum below 2^-6 is 2^-9; from 2^e to 2^(e+1)
 * it is 2^(e-3).  rint rounds ties to even. */
float bdref_round_e4m3(float x)
{
    double a = fabs((double)x);
    if (a != a) return x;
    double q;
    if (a < ldexp(1.0, -6)) {
        q = rint(a / ldexp(1.0, -9)) * ldexp(1.0, -9);
    } else {
        int e;
        frexp(a, &e); /* a = f * 2^e, f in [0.5, 1): 2^(e-1) <= a < 2^e */
        double quantum = ldexp(1.0, (e - 1) - 3);
        q = rint(a / quantum) * quantum;
    }
    if (q > 448.0) q = 448.0;
    return (float)(x < 0 ? -q : q);
}

/* float8 e4m3 scale of a row: the smallest power of two s >= 2^-126 with
 * max|row| <= 448 s (448 is the largest e4m3 value), 1 for an all-zero row.
 * A power of two makes the rescaling v / s exact. */
static float row_scale_e4m3(const float* row, int len)
{
    float m = 0.0f;
    for (int i = 0; i < len; ++i) {
        float v = fabsf(row[i]);
        if (v > m) m = v;
    }
    if (m == 0.0f) return 1.0f;
    int E;
    const double f = frexp((double)m, &E); /* m = f 2^E, f in [0.5, 1) */
    int e = f <= 0.875 ? E - 9 : E - 8;    /* 448 = 0.875 2^9 */
    if (e < -126) e = -126;
    return ldexpf(1.0f, e);
}

void bdref_project_lowp(const float* hist, int32_t n_kp, const float* B, const float* t, int32_t n_bits,
                        int32_t precision, double* resp)
{
    for (int32_t n = 0; n < n_kp; ++n) {
        const float* f = hist + (int64_t)n * 128;
        float sf = precision == 2 ? row_scale_e4m3(f, 128) : 1.0f;
        for (int32_t j = 0; j < n_bits; ++j) {
            const float* b = B + (int64_t)j * 128;
            float sb = precision == 2 ? row_scale_e4m3(b, 128) : 1.0f;
            double acc = 0.0;
            for (int k = 0; k < 128; ++k) {
                double qb, qf;
                if (precision == 1) {
                    qb = bdref_round_bf16(b[k]);
                    qf = bdref_round_bf16(f[k]);
                } else {
                    qb = bdref_round_e4m3(b[k] / sb);
                    qf = bdref_round_e4m3(f[k] / sf);
                }
                acc += qb * qf;
            }
            resp[(int64_t)n * n_bits + j] = (double)sf * (double)sb * acc - (double)t[j];
        }
    }
}

/* ------------------------------------------------------------------ differentiation */

static double patch_box_mean(const float* patch, int cx, int cy, int R)
{
    double sum = 0.0;
    for (int y = cy - R; y <= cy + R; ++y)
        for (int x = cx - R; x <= cx + R; ++x) sum += (double)patch[y * 32 + x];
    return sum / (double)((2 * R + 1) * (2 * R + 1));
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

void bdref_relaxed_bad(const float* patches, int32_t n, const bdref_box_pair* pairs, const double* w1,
                       const double* w2, const double* theta, int32_t n_bits, double beta, double* rho,
                       double* dt, double* m1, double* m2)
{
    for (int32_t i = 0; i < n; ++i) {
        const float* patch = patches + (int64_t)i * 1024;
        for (int32_t j = 0; j < n_bits; ++j) {
            const bdref_box_pair* p = &pairs[j];
            int R = p->radius > 15 ? 15 : p->radius;
            double a = patch_box_mean(patch, clampi(16 + p->x1, R, 31 - R), clampi(16 + p->y1, R, 31 - R), R);
            double b = patch_box_mean(patch, clampi(16 + p->x2, R, 31 - R), clampi(16 + p->y2, R, 31 - R), R);
            double r = theta[j] - (w1[j] * a - w2[j] * b);
            int64_t o = (int64_t)i * n_bits + j;
            if (rho) rho[o] = r;
            if (dt) dt[o] = tanh(beta * r);
            if (m1) m1[o] = a;
            if (m2) m2[o] = b;
        }
    }
}

void bdref_relaxed_hashsift(const double* f, int32_t n, const double* B, const double* t, int32_t n_bits,
                            double beta, double* rho, double* dt)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n_bits; ++j) {
            double r = 0.0;
            for (int k = 0; k < 128; ++k) r += B[(int64_t)j * 128 + k] * f[(int64_t)i * 128 + k];
            r -= t[j];
            int64_t o = (int64_t)i * n_bits + j;
            if (rho) rho[o] = r;
            if (dt) dt[o] = tanh(beta * r);
        }
}

static double sim(const double* x, const double* y, int32_t K)
{
    double s = 0.0;
    for (int32_t k = 0; k < K; ++k) s += x[k] * y[k];
    return s / (double)K;
}

double bdref_trl_hnm(const double* A, const double* P, int32_t n, int32_t n_bits, double tau, int32_t* neg,
                     double* gA, double* gP)
{
    const int32_t K = n_bits;
    if (gA) memset(gA, 0, sizeof(double) * (size_t)n * (size_t)K);
    if (gP) memset(gP, 0, sizeof(double) * (size_t)n * (size_t)K);
    double loss = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        const double* ai = A + (int64_t)i * K;
        const double* pi = P + (int64_t)i * K;
        double best = -INFINITY;
        int32_t choice = 0;
        for (int32_t j = 0; j < n; ++j) { /* row candidates s(a_i, p_j) */
            if (j == i) continue;
            double v = sim(ai, P + (int64_t)j * K, K);
            if (v > best) { best = v; choice = j; }
        }
        for (int32_t j = 0; j < n; ++j) { /* column candidates s(a_j, p_i) */
            if (j == i) continue;
            double v = sim(A + (int64_t)j * K, pi, K);
            if (v > best) { best = v; choice = -1 - j; }
        }
        if (neg) neg[i] = choice;
        double margin = tau - sim(ai, pi, K) + best;
        if (margin <= 0.0 || n < 2) continue;
        loss += margin / (double)n;
        if (!gA || !gP) continue;
        double c = 1.0 / ((double)n * (double)K);
        for (int32_t k = 0; k < K; ++k) { /* d(-s(a_i, p_i)) */
            gA[(int64_t)i * K + k] -= c * pi[k];
            gP[(int64_t)i * K + k] -= c * ai[k];
        }
        if (choice >= 0) { /* d s(a_i, p_j) */
            const double* pj = P + (int64_t)choice * K;
            for (int32_t k = 0; k < K; ++k) {
                gA[(int64_t)i * K + k] += c * pj[k];
                gP[(int64_t)choice * K + k] += c * ai[k];
            }
        } else { /* d s(a_j, p_i) */
            int32_t j = -1 - choice;
            const double* aj = A + (int64_t)j * K;
            for (int32_t k = 0; k < K; ++k) {
                gA[(int64_t)j * K + k] += c * pi[k];
                gP[(int64_t)i * K + k] += c * aj[k];
            }
        }
    }
    return loss;
}

void bdref_relaxed_bad_grad(const double* gD, const double* dt, const double* m1, const double* m2, int32_t n,
                            int32_t n_bits, double beta, double* g_w1, double* g_w2, double* g_theta)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n_bits; ++j) {
            int64_t o = (int64_t)i * n_bits + j;
            double g = gD[o] * beta * (1.0 - dt[o] * dt[o]);
            g_theta[j] += g;
            g_w1[j] -= g * m1[o];
            g_w2[j] += g * m2[o];
        }
}

void bdref_relaxed_hashsift_grad(const double* gD, const double* dt, const double* f, int32_t n, int32_t n_bits,
                                 double beta, double* gB, double* gt)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n_bits; ++j) {
            int64_t o = (int64_t)i * n_bits + j;
            double g = gD[o] * beta * (1.0 - dt[o] * dt[o]);
            gt[j] -= g;
            for (int k = 0; k < 128; ++k) gB[(int64_t)j * 128 + k] += g * f[(int64_t)i * 128 + k];
        }
}

void bdref_hashsift_patch_features(const float* patches, int32_t n, double* f)
{
    bdref_keypoint kp = {15.5f, 15.5f, 1.0f, 0.0f};
    for (int32_t i = 0; i < n; ++i)
        bdref_hashsift_hist(patches + (int64_t)i * 1024, 1, 32, 32, 128, &kp, 1, f + (int64_t)i * 128);
}

/* ------------------------------------------------------------------ feature selection */

/* Sum of the (2r+1)^2 box centred at 16 + u, clamped into the patch. */
static int64_t patch_box_sum_u8(const uint8_t* patch, int ux, int uy, int r)
{
    const int cx = clampi(16 + ux, r, 31 - r), cy = clampi(16 + uy, r, 31 - r);
    int64_t sum = 0;
    for (int y = cy - r; y <= cy + r; ++y)
        for (int x = cx - r; x <= cx + r; ++x) sum += patch[y * 32 + x];
    return sum;
}

int32_t bdref_threshold_bin(const uint8_t* patch, const bdref_box_pair* cand)
{
    const int r = cand->radius > 15 ? 15 : cand->radius;
    const int64_t area = (int64_t)(2 * r + 1) * (2 * r + 1);
    const int64_t s1 = patch_box_sum_u8(patch, cand->x1, cand->y1, r);
    const int64_t s2 = patch_box_sum_u8(patch, cand->x2, cand->y2, r);
    /* (f + 255) * 10 = (10 (s1 - s2) + 2550 area) / area >= 0: exact floor */
    return (int32_t)((10 * (s1 - s2) + 2550 * area) / area);
}

static double trl_term(double tau, int32_t s_ap, int32_t s_an, int ha, int hp, int hn)
{
    const double v = tau - (double)s_ap - (double)(ha * hp) + (double)s_an + (double)(ha * hn);
    return v > 0.0 ? v : 0.0;
}

void bdref_find_threshold(const uint8_t* patches, int32_t n_triplets, const int32_t* s_ap, const int32_t* s_an,
                          double tau, const bdref_box_pair* cands, int32_t n_cands, int32_t* best_bin,
                          double* best_loss)
{
    double* delta = (double*)calloc(BDREF_THRESHOLD_BINS, sizeof(double));
    /* loss with the threshold below every value: every stump is -1 */
    double base = 0.0;
    for (int32_t i = 0; i < n_triplets; ++i) base += trl_term(tau, s_ap[i], s_an[i], -1, -1, -1);
    for (int32_t c = 0; c < n_cands; ++c) {
        memset(delta, 0, BDREF_THRESHOLD_BINS * sizeof(double));
        for (int32_t i = 0; i < n_triplets; ++i) {
            int32_t q[3];
            for (int m = 0; m < 3; ++m) q[m] = bdref_threshold_bin(patches + (int64_t)(3 * i + m) * 1024, &cands[c]);
            /* raise the threshold past the triplet's patches one at a time, in
             * the order of (bin, position in the triplet) */
            int h[3] = {-1, -1, -1};
            int done[3] = {0, 0, 0};
            double prev = trl_term(tau, s_ap[i], s_an[i], h[0], h[1], h[2]);
            for (int step = 0; step < 3; ++step) {
                int next = -1;
                for (int m = 0; m < 3; ++m)
                    if (!done[m] && (next < 0 || q[m] < q[next])) next = m;
                done[next] = 1;
                h[next] = 1;
                const double cur = trl_term(tau, s_ap[i], s_an[i], h[0], h[1], h[2]);
                delta[q[next]] += cur - prev;
                prev = cur;
            }
        }
        /* cumulative sum over the bins in ascending order; first minimum */
        double sum = base, best = INFINITY;
        int32_t bb = -1;
        for (int32_t b = 0; b < BDREF_THRESHOLD_BINS; ++b) {
            sum += delta[b];
            if (sum < best) {
                best = sum;
                bb = b;
            }
        }
        best_bin[c] = bb;
        best_loss[c] = best;
    }
    free(delta);
}

void bdref_hnm_codes(const uint64_t* a_codes, const uint64_t* p_codes, int32_t n, int32_t n_words, int32_t* neg,
                     int32_t* dist_neg, int32_t* dist_pos)
{
    for (int32_t s = 0; s < n; ++s) {
        const uint64_t* as = a_codes + (int64_t)s * n_words;
        const uint64_t* ps = p_codes + (int64_t)s * n_words;
        int32_t jr = -1, jc = -1;
        uint32_t dr = 0, dc = 0;
        /* candidates in cyclic order from s + 1: equal distances keep the first */
        for (int32_t step = 1; step < n; ++step) {
            const int32_t j = (s + step) % n;
            const uint32_t d1 = hamming(as, p_codes + (int64_t)j * n_words, n_words);
            if (jr < 0 || d1 < dr) {
                jr = j;
                dr = d1;
            }
            const uint32_t d2 = hamming(ps, a_codes + (int64_t)j * n_words, n_words);
            if (jc < 0 || d2 < dc) {
                jc = j;
                dc = d2;
            }
        }
        if (dr <= dc) {
            neg[s] = jr;
            dist_neg[s] = (int32_t)dr;
        } else {
            neg[s] = -1 - jc;
            dist_neg[s] = (int32_t)dc;
        }
        dist_pos[s] = (int32_t)hamming(as, ps, n_words);
    }
}

void bdref_select_features(const uint8_t* pool, int32_t n_pairs, const int32_t* samples, int32_t n_sample,
                           const bdref_box_pair* cands, int32_t n_cands, int32_t n_bits, double tau,
                           bdref_box_pair* table, int32_t* chosen, int32_t* chosen_bin, double* round_loss,
                           uint64_t* pool_codes)
{
    const int32_t W = (n_bits + 63) / 64;
    const int32_t n = n_sample;
    uint64_t* codes = (uint64_t*)calloc((size_t)2 * n_pairs * W, sizeof(uint64_t));
    uint64_t* ac = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n * W);
    uint64_t* pc = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n * W);
    int32_t* neg = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* dneg = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* dpos = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* s_ap = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* s_an = (int32_t*)malloc(sizeof(int32_t) * n);
    uint8_t* trip = (uint8_t*)malloc((size_t)3 * n * 1024);
    int32_t* bins = (int32_t*)malloc(sizeof(int32_t) * n_cands);
    double* losses = (double*)malloc(sizeof(double) * n_cands);
    for (int32_t k = 0; k < n_bits; ++k) {
        const int32_t* smp = samples + (int64_t)k * n;
        /* 1. triplets of the sampled pairs by hardest negatives with anchor swap */
        for (int32_t s = 0; s < n; ++s) {
            memcpy(ac + (int64_t)s * W, codes + (int64_t)(2 * smp[s]) * W, sizeof(uint64_t) * W);
            memcpy(pc + (int64_t)s * W, codes + (int64_t)(2 * smp[s] + 1) * W, sizeof(uint64_t) * W);
        }
        bdref_hnm_codes(ac, pc, n, W, neg, dneg, dpos);
        for (int32_t s = 0; s < n; ++s) {
            int32_t anc, pos, ngp;
            if (neg[s] >= 0) {
                anc = 2 * smp[s];
                pos = 2 * smp[s] + 1;
                ngp = 2 * smp[neg[s]] + 1;
            } else {
                anc = 2 * smp[s] + 1;
                pos = 2 * smp[s];
                ngp = 2 * smp[-1 - neg[s]];
            }
            memcpy(trip + (int64_t)(3 * s) * 1024, pool + (int64_t)anc * 1024, 1024);
            memcpy(trip + (int64_t)(3 * s + 1) * 1024, pool + (int64_t)pos * 1024, 1024);
            memcpy(trip + (int64_t)(3 * s + 2) * 1024, pool + (int64_t)ngp * 1024, 1024);
            s_ap[s] = k - 2 * dpos[s];
            s_an[s] = k - 2 * dneg[s];
        }
        /* 2. the best threshold of every candidate, then the best candidate */
        const bdref_box_pair* ck = cands + (int64_t)k * n_cands;
        bdref_find_threshold(trip, n, s_ap, s_an, tau, ck, n_cands, bins, losses);
        int32_t best = 0;
        for (int32_t c = 1; c < n_cands; ++c)
            if (losses[c] < losses[best]) best = c;
        const int r = ck[best].radius > 15 ? 15 : ck[best].radius;
        table[k] = ck[best];
        table[k].threshold = (float)((double)(bins[best] + 1 - 2550) / 10.0 - 1.0 / (20.0 * (2 * r + 1) * (2 * r + 1)));
        if (chosen) chosen[k] = best;
        if (chosen_bin) chosen_bin[k] = bins[best];
        if (round_loss) round_loss[k] = losses[best];
        /* 3. the new stump becomes bit k of every pool patch */
        for (int32_t x = 0; x < 2 * n_pairs; ++x)
            if (bdref_threshold_bin(pool + (int64_t)x * 1024, &ck[best]) <= bins[best])
                codes[(int64_t)x * W + k / 64] |= 1ull << (k % 64);
    }
    if (pool_codes) memcpy(pool_codes, codes, sizeof(uint64_t) * (size_t)2 * n_pairs * W);
    free(codes);
    free(ac);
    free(pc);
    free(neg);
    free(dneg);
    free(dpos);
    free(s_ap);
    free(s_an);
    free(trip);
    free(bins);
    free(losses);
}

/* ------------------------------------------------------------------ training augmentation */

static double patch_at(const float* p, int x, int y)
{
    x = clampi(x, 0, 31);
    y = clampi(y, 0, 31);
    return (double)p[y * 32 + x];
}

void bdref_augment_patches(const float* src, int32_t n, const double* params, const float* noise, float* dst)
{
    double warp[1024], tmp[1024];
    for (int32_t k = 0; k < n; ++k) {
        const float* s = src + (int64_t)k * 1024;
        const double* pr = params + (int64_t)k * 5;
        const double ca = cos(pr[0]), sa = sin(pr[0]), sc = pr[1];
        /* 1. rotation and scale about the patch centre, bilinear */
        for (int i = 0; i < 32; ++i)
            for (int j = 0; j < 32; ++j) {
                const double ux = j - 15.5, uy = i - 15.5;
                const double px = 15.5 + sc * (ca * ux - sa * uy);
                const double py = 15.5 + sc * (sa * ux + ca * uy);
                const double x0 = floor(px), y0 = floor(py);
                const double fx = px - x0, fy = py - y0;
                const int xi = (int)x0, yi = (int)y0;
                const double top = patch_at(s, xi, yi) + fx * (patch_at(s, xi + 1, yi) - patch_at(s, xi, yi));
                const double bot =
                    patch_at(s, xi, yi + 1) + fx * (patch_at(s, xi + 1, yi + 1) - patch_at(s, xi, yi + 1));
                warp[i * 32 + j] = top + fy * (bot - top);
            }
        /* 2. separable Gaussian blur */
        const double sigma = pr[4] > 4.0 ? 4.0 : pr[4];
        if (sigma > 0.0) {
            const int R = (int)ceil(3.0 * sigma);
            double w[64], wsum = 0.0;
            for (int d = -R; d <= R; ++d) wsum += (w[d + R] = exp(-(double)(d * d) / (2.0 * sigma * sigma)));
            for (int d = 0; d <= 2 * R; ++d) w[d] /= wsum;
            for (int i = 0; i < 32; ++i)
                for (int j = 0; j < 32; ++j) {
                    double acc = 0.0;
                    for (int d = -R; d <= R; ++d) acc += w[d + R] * warp[i * 32 + clampi(j + d, 0, 31)];
                    tmp[i * 32 + j] = acc;
                }
            for (int i = 0; i < 32; ++i)
                for (int j = 0; j < 32; ++j) {
                    double acc = 0.0;
                    for (int d = -R; d <= R; ++d) acc += w[d + R] * tmp[clampi(i + d, 0, 31) * 32 + j];
                    warp[i * 32 + j] = acc;
                }
        }
        /* 3-5. illumination, noise, clipping */
        for (int e = 0; e < 1024; ++e) {
            double v = pr[2] * warp[e] + pr[3] + (double)noise[(int64_t)k * 1024 + e];
            v = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            dst[(int64_t)k * 1024 + e] = (float)v;
        }
    }
}
