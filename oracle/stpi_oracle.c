/*
 * FP64 CPU oracle for the space-time power iteration (TEST INFRASTRUCTURE).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file. It shares no code, header, table or constant with the HIP
 * library: it is a plain, slow restatement of the method's definitions.
 *
 * Operator (Sec. 3, Eq. 2 with alpha = 0 and the unary feature s^p taken as f;
 * Eq. 4 for the neighbourhood sum; first convolution term of Eq. 7):
 *
 *   A_ij = f_i * f_j * G_ij,
 *   G_ij = exp(-dt^2/(2 st^2)) * exp(-dy^2/(2 ss^2)) * exp(-dx^2/(2 ss^2))
 *          when |dt| <= r_t, |dy| <= r_s, |dx| <= r_s and j lies inside the
 *          T x H x W volume, 0 otherwise (unnormalised, G_ii = 1).
 *
 *   (A x)_i = f_i * sum_{j in N(i)} G_ij f_j x_j      (direct 3D box loop)
 *
 * Nothing here is separable, blocked or reordered: each output is the full
 * (2r_t+1)(2r_s+1)^2 neighbourhood sum in double, in (dt, dy, dx) order.
 *
 * The warm-start network helpers below are the plain definition of a 'same'
 * 3x3x3 convolution with zero padding (forward and its exact derivatives).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* G(dt, dy, dx): product of three one-dimensional Gaussians, peak value 1. */
static double affinity_weight(int dt, int dy, int dx, double sigma_s, double sigma_t) {
    double et = exp(-(double)(dt * dt) / (2.0 * sigma_t * sigma_t));
    double ey = exp(-(double)(dy * dy) / (2.0 * sigma_s * sigma_s));
    double ex = exp(-(double)(dx * dx) / (2.0 * sigma_s * sigma_s));
    return et * ey * ex;
}

static double *weight_box(double sigma_s, double sigma_t, int r_s, int r_t) {
    int nt = 2 * r_t + 1, ns = 2 * r_s + 1;
    double *w = (double *)malloc(sizeof(double) * (size_t)nt * ns * ns);
    if (!w) return NULL;
    for (int dt = -r_t; dt <= r_t; ++dt)
        for (int dy = -r_s; dy <= r_s; ++dy)
            for (int dx = -r_s; dx <= r_s; ++dx)
                w[((size_t)(dt + r_t) * ns + (dy + r_s)) * ns + (dx + r_s)] =
                    affinity_weight(dt, dy, dx, sigma_s, sigma_t);
    return w;
}

/* sum_{j in N(i)} G_ij * f_j * x_j for voxel i = (t, y, x). */
static double neighbourhood_sum(int T, int H, int W, const double *f, const double *xv,
                                const double *w, int r_s, int r_t, int t, int y, int x) {
    int ns = 2 * r_s + 1;
    double acc = 0.0;
    for (int dt = -r_t; dt <= r_t; ++dt) {
        int tt = t + dt;
        if (tt < 0 || tt >= T) continue;
        for (int dy = -r_s; dy <= r_s; ++dy) {
            int yy = y + dy;
            if (yy < 0 || yy >= H) continue;
            const double *wrow = w + ((size_t)(dt + r_t) * ns + (dy + r_s)) * ns + r_s;
            size_t base = ((size_t)tt * H + yy) * W;
            for (int dx = -r_s; dx <= r_s; ++dx) {
                int xx = x + dx;
                if (xx < 0 || xx >= W) continue;
                acc += wrow[dx] * f[base + xx] * xv[base + xx];
            }
        }
    }
    return acc;
}

/* z = A x over the whole volume. Returns 0 on success, 1 on bad arguments. */
int oracle_apply(int T, int H, int W, const double *f, const double *x,
                 double sigma_s, double sigma_t, int r_s, int r_t, double *z) {
    if (T < 1 || H < 1 || W < 1 || r_s < 0 || r_t < 0 || !(sigma_s > 0) || !(sigma_t > 0))
        return 1;
    double *w = weight_box(sigma_s, sigma_t, r_s, r_t);
    if (!w) return 1;
    long rows = (long)T * H;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        int t = (int)(row / H), y = (int)(row % H);
        for (int xi = 0; xi < W; ++xi) {
            size_t i = (size_t)row * W + xi;
            z[i] = f[i] * neighbourhood_sum(T, H, W, f, x, w, r_s, r_t, t, y, xi);
        }
    }
    free(w);
    return 0;
}

/* (A x)_i for the listed flat indices only (sampled parity at full size). */
int oracle_apply_at(int T, int H, int W, const double *f, const double *x,
                    double sigma_s, double sigma_t, int r_s, int r_t,
                    const int64_t *idx, int64_t n_idx, double *out) {
    if (T < 1 || H < 1 || W < 1 || r_s < 0 || r_t < 0 || !(sigma_s > 0) || !(sigma_t > 0))
        return 1;
    double *w = weight_box(sigma_s, sigma_t, r_s, r_t);
    if (!w) return 1;
    int64_t N = (int64_t)T * H * W;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < n_idx; ++k) {
        int64_t i = idx[k];
        if (i < 0 || i >= N) { bad |= 1; out[k] = NAN; continue; }
        int t = (int)(i / ((int64_t)H * W));
        int y = (int)((i / W) % H);
        int xi = (int)(i % W);
        out[k] = f[i] * neighbourhood_sum(T, H, W, f, x, w, r_s, r_t, t, y, xi);
    }
    free(w);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Full SFSeg operator (Sec. 3: Eq. 2, its first-order Taylor affinity, and the
 * power-iteration update of Eq. 5-7). With the unary map s (already raised to
 * the power p) and the pairwise feature f,
 *
 *   M_ij = s_i s_j [1 - alpha (f_i - f_j)^2] G_ij                  (Eq. 2)
 *
 * and the update as Eq. 7 writes it (Eq. 5 without its leading alpha) is
 *
 *   z_i = (M x)_i / alpha = s_i sum_{j in N(i)} s_j [1/alpha - (f_i - f_j)^2] G_ij x_j.
 *
 * Direct 3D box loop in double, in (dt, dy, dx) order, like oracle_apply.
 * ------------------------------------------------------------------------- */
static double sfseg_sum(int T, int H, int W, const double *s, const double *f, const double *xv, double ainv,
                        const double *w, int r_s, int r_t, int t, int y, int x) {
    int ns = 2 * r_s + 1;
    double fi = f[((size_t)t * H + y) * W + x];
    double acc = 0.0;
    for (int dt = -r_t; dt <= r_t; ++dt) {
        int tt = t + dt;
        if (tt < 0 || tt >= T) continue;
        for (int dy = -r_s; dy <= r_s; ++dy) {
            int yy = y + dy;
            if (yy < 0 || yy >= H) continue;
            const double *wrow = w + ((size_t)(dt + r_t) * ns + (dy + r_s)) * ns + r_s;
            size_t base = ((size_t)tt * H + yy) * W;
            for (int dx = -r_s; dx <= r_s; ++dx) {
                int xx = x + dx;
                if (xx < 0 || xx >= W) continue;
                double d = fi - f[base + xx];
                acc += s[base + xx] * (ainv - d * d) * wrow[dx] * xv[base + xx];
            }
        }
    }
    return acc;
}

int oracle_sfseg_apply(int T, int H, int W, const double *s, const double *f, const double *x, double alpha,
                       double sigma_s, double sigma_t, int r_s, int r_t, double *z) {
    if (T < 1 || H < 1 || W < 1 || r_s < 0 || r_t < 0 || !(sigma_s > 0) || !(sigma_t > 0) || !(alpha > 0))
        return 1;
    double *w = weight_box(sigma_s, sigma_t, r_s, r_t);
    if (!w) return 1;
    double ainv = 1.0 / alpha;
    long rows = (long)T * H;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        int t = (int)(row / H), y = (int)(row % H);
        for (int xi = 0; xi < W; ++xi) {
            size_t i = (size_t)row * W + xi;
            z[i] = s[i] * sfseg_sum(T, H, W, s, f, x, ainv, w, r_s, r_t, t, y, xi);
        }
    }
    free(w);
    return 0;
}

int oracle_sfseg_apply_at(int T, int H, int W, const double *s, const double *f, const double *x, double alpha,
                          double sigma_s, double sigma_t, int r_s, int r_t, const int64_t *idx, int64_t n_idx,
                          double *out) {
    if (T < 1 || H < 1 || W < 1 || r_s < 0 || r_t < 0 || !(sigma_s > 0) || !(sigma_t > 0) || !(alpha > 0))
        return 1;
    double *w = weight_box(sigma_s, sigma_t, r_s, r_t);
    if (!w) return 1;
    double ainv = 1.0 / alpha;
    int64_t N = (int64_t)T * H * W;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < n_idx; ++k) {
        int64_t i = idx[k];
        if (i < 0 || i >= N) { bad |= 1; out[k] = NAN; continue; }
        int t = (int)(i / ((int64_t)H * W));
        int y = (int)((i / W) % H);
        int xi = (int)(i % W);
        out[k] = s[i] * sfseg_sum(T, H, W, s, f, x, ainv, w, r_s, r_t, t, y, xi);
    }
    free(w);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Exact pairwise affinity (Sec. 3, Eq. 1, before the Taylor approximation):
 *
 *   E_ij = s_i s_j exp(-alpha (f_i - f_j)^2) G_ij,   z = E x,
 *
 * direct 3D box loop in double, (dt, dy, dx) order.
 * ------------------------------------------------------------------------- */
int oracle_exp_apply(int T, int H, int W, const double *s, const double *f, const double *x, double alpha,
                     double sigma_s, double sigma_t, int r_s, int r_t, double *z) {
    if (T < 1 || H < 1 || W < 1 || r_s < 0 || r_t < 0 || !(sigma_s > 0) || !(sigma_t > 0) || !(alpha >= 0))
        return 1;
    double *w = weight_box(sigma_s, sigma_t, r_s, r_t);
    if (!w) return 1;
    int ns = 2 * r_s + 1;
    long rows = (long)T * H;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        int t = (int)(row / H), y = (int)(row % H);
        for (int xi = 0; xi < W; ++xi) {
            size_t i = (size_t)row * W + xi;
            double acc = 0.0;
            for (int dt = -r_t; dt <= r_t; ++dt) {
                int tt = t + dt;
                if (tt < 0 || tt >= T) continue;
                for (int dy = -r_s; dy <= r_s; ++dy) {
                    int yy = y + dy;
                    if (yy < 0 || yy >= H) continue;
                    const double *wrow = w + ((size_t)(dt + r_t) * ns + (dy + r_s)) * ns + r_s;
                    size_t base = ((size_t)tt * H + yy) * W;
                    for (int dx = -r_s; dx <= r_s; ++dx) {
                        int xx = xi + dx;
                        if (xx < 0 || xx >= W) continue;
                        double d = f[i] - f[base + xx];
                        acc += s[base + xx] * exp(-alpha * d * d) * wrow[dx] * x[base + xx];
                    }
                }
            }
            z[i] = s[i] * acc;
        }
    }
    free(w);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Warm-start network: 'same' 3x3x3 convolution, zero padding, bias.
 * in  [Cin][T][H][W], wgt [Cout][Cin][3][3][3], bias [Cout], out [Cout][T][H][W]
 *   out[o,t,y,x] = bias[o] + sum_{i,a,b,c} wgt[o,i,a,b,c] * in[i, t+a-1, y+b-1, x+c-1]
 * ------------------------------------------------------------------------- */
int oracle_conv3d_fwd(int Cin, int Cout, int T, int H, int W, const double *in,
                      const double *wgt, const double *bias, double *out) {
    if (Cin < 1 || Cout < 1 || T < 1 || H < 1 || W < 1) return 1;
    size_t N = (size_t)T * H * W;
    long rows = (long)Cout * T * H;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        int o = (int)(row / ((long)T * H));
        int t = (int)((row / H) % T);
        int y = (int)(row % H);
        for (int x = 0; x < W; ++x) {
            double acc = bias ? bias[o] : 0.0;
            for (int i = 0; i < Cin; ++i)
                for (int a = 0; a < 3; ++a) {
                    int tt = t + a - 1;
                    if (tt < 0 || tt >= T) continue;
                    for (int b = 0; b < 3; ++b) {
                        int yy = y + b - 1;
                        if (yy < 0 || yy >= H) continue;
                        for (int c = 0; c < 3; ++c) {
                            int xx = x + c - 1;
                            if (xx < 0 || xx >= W) continue;
                            acc += wgt[(((size_t)o * Cin + i) * 3 + a) * 9 + b * 3 + c] *
                                   in[(size_t)i * N + ((size_t)tt * H + yy) * W + xx];
                        }
                    }
                }
            out[(size_t)o * N + ((size_t)t * H + y) * W + x] = acc;
        }
    }
    return 0;
}

/* Given g_out = dL/dout: g_in = dL/din (may be NULL), g_w = dL/dwgt, g_b = dL/dbias
 * (both overwritten, may be NULL). */
int oracle_conv3d_bwd(int Cin, int Cout, int T, int H, int W, const double *in,
                      const double *wgt, const double *g_out, double *g_in,
                      double *g_w, double *g_b) {
    if (Cin < 1 || Cout < 1 || T < 1 || H < 1 || W < 1) return 1;
    size_t N = (size_t)T * H * W;
    if (g_in) {
        /* g_in[i, p] = sum_{o, taps} wgt[o,i,tap] * g_out[o, p - tap + 1] */
        long rows = (long)Cin * T * H;
#pragma omp parallel for schedule(static)
        for (long row = 0; row < rows; ++row) {
            int i = (int)(row / ((long)T * H));
            int t = (int)((row / H) % T);
            int y = (int)(row % H);
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int o = 0; o < Cout; ++o)
                    for (int a = 0; a < 3; ++a) {
                        int tt = t - a + 1;
                        if (tt < 0 || tt >= T) continue;
                        for (int b = 0; b < 3; ++b) {
                            int yy = y - b + 1;
                            if (yy < 0 || yy >= H) continue;
                            for (int c = 0; c < 3; ++c) {
                                int xx = x - c + 1;
                                if (xx < 0 || xx >= W) continue;
                                acc += wgt[(((size_t)o * Cin + i) * 3 + a) * 9 + b * 3 + c] *
                                       g_out[(size_t)o * N + ((size_t)tt * H + yy) * W + xx];
                            }
                        }
                    }
                g_in[(size_t)i * N + ((size_t)t * H + y) * W + x] = acc;
            }
        }
    }
    if (g_w) {
        int ntap = Cout * Cin * 27;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ntap; ++k) {
            int o = k / (Cin * 27), i = (k / 27) % Cin, tap = k % 27;
            int a = tap / 9, b = (tap / 3) % 3, c = tap % 3;
            double acc = 0.0;
            for (int t = 0; t < T; ++t) {
                int tt = t + a - 1;
                if (tt < 0 || tt >= T) continue;
                for (int y = 0; y < H; ++y) {
                    int yy = y + b - 1;
                    if (yy < 0 || yy >= H) continue;
                    for (int x = 0; x < W; ++x) {
                        int xx = x + c - 1;
                        if (xx < 0 || xx >= W) continue;
                        acc += g_out[(size_t)o * N + ((size_t)t * H + y) * W + x] *
                               in[(size_t)i * N + ((size_t)tt * H + yy) * W + xx];
                    }
                }
            }
            g_w[k] = acc;
        }
    }
    if (g_b) {
        for (int o = 0; o < Cout; ++o) {
            double acc = 0.0;
            for (size_t p = 0; p < N; ++p) acc += g_out[(size_t)o * N + p];
            g_b[o] = acc;
        }
    }
    return 0;
}
