/*
 * Plain FP64 CPU oracle of the surrogate network's operations: 3x3x3
 * convolution (forward, gradient with respect to the input, gradient with
 * respect to the weights and bias), 2x average pooling, 2x nearest
 * upsampling, leaky ReLU, mean-squared error, the Adam update, and the
 * semi-Lagrangian phase transport and the projective time step that serve as
 * jump baselines.
 *
 * TEST INFRASTRUCTURE ONLY: for the tests and the smoke check; shares no code
 * with the GPU library.
 *
 * Tensors are channels-last: x[((n*D + d)*H + h)*W + w][c].  Convolution
 * weights are w[t][co][ci] with tap t = (a+1)*9 + (b+1)*3 + (c+1) for the
 * offset (a, b, c) in (d, h, w); zero padding of one cell, stride one:
 *   y[v][co] = bias[co] + sum_t sum_ci x[v + offset(t)][ci] w[t][co][ci].
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

static inline int64_t vox(int n, int d, int h, int w, int D, int H, int W)
{
    return (((int64_t)n * D + d) * H + h) * W + w;
}

void orc_conv3d_fwd(const double *x, int N, int D, int H, int W, int Ci, const double *wt,
                    const double *bias, int Co, double *y)
{
    for (int n = 0; n < N; ++n)
        for (int d = 0; d < D; ++d)
            for (int h = 0; h < H; ++h)
                for (int w = 0; w < W; ++w) {
                    double *yo = y + vox(n, d, h, w, D, H, W) * Co;
                    for (int co = 0; co < Co; ++co) yo[co] = bias ? bias[co] : 0.0;
                    for (int a = -1; a <= 1; ++a)
                        for (int b = -1; b <= 1; ++b)
                            for (int c = -1; c <= 1; ++c) {
                                const int dd = d + a, hh = h + b, ww = w + c;
                                if (dd < 0 || dd >= D || hh < 0 || hh >= H || ww < 0 || ww >= W) continue;
                                const int t = (a + 1) * 9 + (b + 1) * 3 + (c + 1);
                                const double *xi = x + vox(n, dd, hh, ww, D, H, W) * Ci;
                                for (int co = 0; co < Co; ++co) {
                                    const double *wr = wt + ((int64_t)t * Co + co) * Ci;
                                    double s = 0.0;
                                    for (int ci = 0; ci < Ci; ++ci) s += xi[ci] * wr[ci];
                                    yo[co] += s;
                                }
                            }
                }
}

/* dx[v][ci] = sum_t sum_co dy[v - offset(t)][co] w[t][co][ci] */
void orc_conv3d_bwd_data(const double *dy, int N, int D, int H, int W, int Co, const double *wt, int Ci,
                         double *dx)
{
    memset(dx, 0, sizeof(double) * (size_t)N * D * H * W * Ci);
    for (int n = 0; n < N; ++n)
        for (int d = 0; d < D; ++d)
            for (int h = 0; h < H; ++h)
                for (int w = 0; w < W; ++w) {
                    const double *g = dy + vox(n, d, h, w, D, H, W) * Co;
                    for (int a = -1; a <= 1; ++a)
                        for (int b = -1; b <= 1; ++b)
                            for (int c = -1; c <= 1; ++c) {
                                const int dd = d + a, hh = h + b, ww = w + c;
                                if (dd < 0 || dd >= D || hh < 0 || hh >= H || ww < 0 || ww >= W) continue;
                                const int t = (a + 1) * 9 + (b + 1) * 3 + (c + 1);
                                double *xo = dx + vox(n, dd, hh, ww, D, H, W) * Ci;
                                for (int co = 0; co < Co; ++co) {
                                    const double *wr = wt + ((int64_t)t * Co + co) * Ci;
                                    for (int ci = 0; ci < Ci; ++ci) xo[ci] += g[co] * wr[ci];
                                }
                            }
                }
}

/* dw[t][co][ci] = sum_v dy[v][co] x[v + offset(t)][ci];  db[co] = sum_v dy[v][co] */
void orc_conv3d_bwd_weight(const double *x, const double *dy, int N, int D, int H, int W, int Ci, int Co,
                           double *dw, double *db)
{
    memset(dw, 0, sizeof(double) * 27 * (size_t)Co * Ci);
    if (db) memset(db, 0, sizeof(double) * Co);
    for (int n = 0; n < N; ++n)
        for (int d = 0; d < D; ++d)
            for (int h = 0; h < H; ++h)
                for (int w = 0; w < W; ++w) {
                    const double *g = dy + vox(n, d, h, w, D, H, W) * Co;
                    if (db)
                        for (int co = 0; co < Co; ++co) db[co] += g[co];
                    for (int a = -1; a <= 1; ++a)
                        for (int b = -1; b <= 1; ++b)
                            for (int c = -1; c <= 1; ++c) {
                                const int dd = d + a, hh = h + b, ww = w + c;
                                if (dd < 0 || dd >= D || hh < 0 || hh >= H || ww < 0 || ww >= W) continue;
                                const int t = (a + 1) * 9 + (b + 1) * 3 + (c + 1);
                                const double *xi = x + vox(n, dd, hh, ww, D, H, W) * Ci;
                                for (int co = 0; co < Co; ++co) {
                                    double *wr = dw + ((int64_t)t * Co + co) * Ci;
                                    for (int ci = 0; ci < Ci; ++ci) wr[ci] += g[co] * xi[ci];
                                }
                            }
                }
}

/* y = mean of each 2x2x2 block (D, H, W even) */
void orc_pool2(const double *x, int N, int D, int H, int W, int C, double *y)
{
    const int d2 = D / 2, h2 = H / 2, w2 = W / 2;
    for (int n = 0; n < N; ++n)
        for (int d = 0; d < d2; ++d)
            for (int h = 0; h < h2; ++h)
                for (int w = 0; w < w2; ++w)
                    for (int c = 0; c < C; ++c) {
                        double s = 0.0;
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b)
                                for (int e = 0; e < 2; ++e)
                                    s += x[vox(n, 2 * d + a, 2 * h + b, 2 * w + e, D, H, W) * C + c];
                        y[vox(n, d, h, w, d2, h2, w2) * C + c] = s / 8.0;
                    }
}

/* y[2d+a][2h+b][2w+e] = x[d][h][w]  (D, H, W of the coarse input) */
void orc_up2(const double *x, int N, int D, int H, int W, int C, double *y)
{
    for (int n = 0; n < N; ++n)
        for (int d = 0; d < 2 * D; ++d)
            for (int h = 0; h < 2 * H; ++h)
                for (int w = 0; w < 2 * W; ++w)
                    for (int c = 0; c < C; ++c)
                        y[vox(n, d, h, w, 2 * D, 2 * H, 2 * W) * C + c] = x[vox(n, d / 2, h / 2, w / 2, D, H, W) * C + c];
}

/* leaky ReLU: y = x (x > 0), slope * x otherwise */
void orc_leaky(const double *x, size_t n, double slope, double *y)
{
    for (size_t i = 0; i < n; ++i) y[i] = x[i] > 0.0 ? x[i] : slope * x[i];
}

/* mean squared error and its gradient with respect to pred */
double orc_mse(const double *pred, const double *target, size_t n, double *grad)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double d = pred[i] - target[i];
        s += d * d;
        if (grad) grad[i] = 2.0 * d / (double)n;
    }
    return s / (double)n;
}

/* Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t >= 1. */
void orc_adam(double *p, const double *g, double *m, double *v, size_t n, double lr, double b1, double b2,
              double eps, int t)
{
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (size_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Physics baseline of a jump of K steps on a box of states (5 channels per
 * voxel, channels last: phi, u_x, u_y, u_z, p; voxel v = x + bx (y + by z)):
 * semi-Lagrangian transport of phi by the local velocity,
 *   phi'(x) = phi(x - K u(x))   (trilinear interpolation, the departure
 *                                point clamped to the box),
 * with u and p carried over unchanged.  count boxes one after another.   */
void orc_advect_phase(const double *state, int count, int bx, int by, int bz, double K, double *out)
{
    const int64_t V = (int64_t)bx * by * bz;
    for (int n = 0; n < count; ++n) {
        const double *s = state + (int64_t)n * V * 5;
        double *o = out + (int64_t)n * V * 5;
        for (int z = 0; z < bz; ++z)
            for (int y = 0; y < by; ++y)
                for (int x = 0; x < bx; ++x) {
                    const int64_t v = x + (int64_t)bx * (y + (int64_t)by * z);
                    const double *sv = s + v * 5;
                    double p[3] = {x - K * sv[1], y - K * sv[2], z - K * sv[3]};
                    const int ext[3] = {bx, by, bz};
                    int lo[3], hi[3];
                    double f[3];
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] < 0.0) p[a] = 0.0;
                        if (p[a] > ext[a] - 1) p[a] = ext[a] - 1;
                        lo[a] = (int)floor(p[a]);
                        hi[a] = lo[a] + 1 < ext[a] ? lo[a] + 1 : lo[a];
                        f[a] = p[a] - lo[a];
                    }
                    double phi = 0.0;
                    for (int cz = 0; cz < 2; ++cz)
                        for (int cy = 0; cy < 2; ++cy)
                            for (int cx = 0; cx < 2; ++cx) {
                                const int xx = cx ? hi[0] : lo[0], yy = cy ? hi[1] : lo[1], zz = cz ? hi[2] : lo[2];
                                const double wgt = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) *
                                                   (cz ? f[2] : 1.0 - f[2]);
                                phi += wgt * s[(xx + (int64_t)bx * (yy + (int64_t)by * zz)) * 5];
                            }
                    o[v * 5] = phi;
                    for (int k = 1; k < 5; ++k) o[v * 5 + k] = sv[k];
                }
    }
}

/* Co-moving baseline of a jump on boxes of states (layout as above): the
 * whole state is translated by the box's displacement d_n = shift[4n..4n+2],
 *   s'(x) = s(x - d_n)   (trilinear interpolation of every channel, the
 *                         departure point clamped to the box),
 * and the velocity channels are multiplied by f_n = shift[4n+3].  A bubble
 * rising at a constant speed U is steady in its own frame, so d = K U,
 * f = 1 is the exact jump of K steps in that limit.                       */
void orc_shift_boxes(const double *state, int count, int bx, int by, int bz, const double *shift, double *out)
{
    const int64_t V = (int64_t)bx * by * bz;
    const int ext[3] = {bx, by, bz};
    for (int n = 0; n < count; ++n) {
        const double *s = state + (int64_t)n * V * 5;
        double *o = out + (int64_t)n * V * 5;
        for (int z = 0; z < bz; ++z)
            for (int y = 0; y < by; ++y)
                for (int x = 0; x < bx; ++x) {
                    const int64_t v = x + (int64_t)bx * (y + (int64_t)by * z);
                    double p[3] = {x - shift[4 * n], y - shift[4 * n + 1], z - shift[4 * n + 2]};
                    int lo[3], hi[3];
                    double f[3];
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] < 0.0) p[a] = 0.0;
                        if (p[a] > ext[a] - 1) p[a] = ext[a] - 1;
                        lo[a] = (int)floor(p[a]);
                        hi[a] = lo[a] + 1 < ext[a] ? lo[a] + 1 : lo[a];
                        f[a] = p[a] - lo[a];
                    }
                    for (int k = 0; k < 5; ++k) {
                        double acc = 0.0;
                        for (int cz = 0; cz < 2; ++cz)
                            for (int cy = 0; cy < 2; ++cy)
                                for (int cx = 0; cx < 2; ++cx) {
                                    const int xx = cx ? hi[0] : lo[0], yy = cy ? hi[1] : lo[1];
                                    const int zz = cz ? hi[2] : lo[2];
                                    const double wgt = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) *
                                                       (cz ? f[2] : 1.0 - f[2]);
                                    acc += wgt * s[(xx + (int64_t)bx * (yy + (int64_t)by * zz)) * 5 + k];
                                }
                        o[v * 5 + k] = (k >= 1 && k <= 3) ? acc * shift[4 * n + 3] : acc;
                    }
                }
    }
}

/* Gas-indicator moments of boxes of states: chi = (phi_heavy - phi) /
 * (phi_heavy - phi_light) clipped to [0, 1] (the gas indicator of the
 * statistics, whose centroid and chi-weighted u_y define the rise of a
 * bubble); out[8n + k] = sum chi, sum chi x, sum chi y, sum chi z,
 * sum chi u_x, sum chi u_y, sum chi u_z, 0 over box n.                   */
void orc_box_moments(const double *state, int count, int bx, int by, int bz, double pheavy, double plight,
                     double *out)
{
    const int64_t V = (int64_t)bx * by * bz;
    for (int n = 0; n < count; ++n) {
        double *o = out + 8 * n;
        for (int k = 0; k < 8; ++k) o[k] = 0.0;
        for (int z = 0; z < bz; ++z)
            for (int y = 0; y < by; ++y)
                for (int x = 0; x < bx; ++x) {
                    const double *sv = state + ((int64_t)n * V + x + (int64_t)bx * (y + (int64_t)by * z)) * 5;
                    double chi = (pheavy - sv[0]) / (pheavy - plight);
                    if (chi < 0.0) chi = 0.0;
                    if (chi > 1.0) chi = 1.0;
                    o[0] += chi;
                    o[1] += chi * x;
                    o[2] += chi * y;
                    o[3] += chi * z;
                    o[4] += chi * sv[1];
                    o[5] += chi * sv[2];
                    o[6] += chi * sv[3];
                }
    }
}

/* Projective (coarse) time step of the macroscopic fields (Gear and
 * Kevrekidis, "Projective methods for stiff differential equations", SIAM
 * J. Sci. Comput. 24, 2003): with s the fields now and s_prev the fields m
 * LBM steps earlier, the fields K steps ahead are extrapolated linearly,
 *   s' = s + (K/m) (s - s_prev),
 * channel by channel for n points.  Element (i, k) of a field set sits at
 * f[k * cs + i * vs] (planar: cs = n, vs = 1; channels last: cs = 1,
 * vs = 5); channels are (phi, u_x, u_y, u_z, p).  phi' is clipped to
 * [phi_lo, phi_hi]; with u_by_phase == 1 the velocity increment is weighted
 * by the heavy-phase fraction q = clamp((phi - phi_lo)/(phi_hi - phi_lo),
 * 0, 1) of the current phi, with u_by_phase == 2 by clamp(10 q - 9, 0, 1)
 * (the bulk of the heavy phase only, none within the interface); with
 * phi_step == 0 phi is carried over (then only clipped), with p_step == 0
 * the pressure.                                                          */
void orc_projective_step(const double *s, const double *s_prev, int64_t n, int64_t cs, int64_t vs, double ratio,
                         double phi_lo, double phi_hi, int u_by_phase, int phi_step, int p_step, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        const double phi = s[i * vs], dphi = phi - s_prev[i * vs];
        double q = (phi - phi_lo) / (phi_hi - phi_lo);
        q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
        double np = phi_step ? phi + ratio * dphi : phi;
        np = np < phi_lo ? phi_lo : (np > phi_hi ? phi_hi : np);
        out[i * vs] = np;
        for (int k = 1; k <= 3; ++k) {
            const double v = s[k * cs + i * vs], dv = v - s_prev[k * cs + i * vs];
            double wq = 1.0;
            if (u_by_phase == 1) wq = q;
            if (u_by_phase == 2) wq = 10.0 * q - 9.0 < 0.0 ? 0.0 : 10.0 * q - 9.0;
            out[k * cs + i * vs] = v + wq * ratio * dv;
        }
        const double p = s[4 * cs + i * vs];
        out[4 * cs + i * vs] = p_step ? p + ratio * (p - s_prev[4 * cs + i * vs]) : p;
    }
}

/* Mass projection of a phase field after a jump (part of the learned
 * fast-forward, not of the paper's method).  The jump may change sum(phi),
 * which the scheme itself conserves exactly (Section 3.1); the projection
 * restores it by moving phi only inside the interface:
 *   q   = clamp((phi - phi_min) / (phi_max - phi_min), 0, 1),
 *   w   = 4 q (1 - q)               (0 in both bulk phases, 1 at q = 1/2),
 *   c   = (target - sum phi) / sum w  (0 if sum w = 0),
 *   phi' = phi + c w,
 * with both sums over the fluid cells of an nx*ny*nz grid (x fastest);
 * with walls_y the rows y = 0 and ny-1 are solid: they take no part in the
 * sums and are left unchanged.  Plain FP64, serial in storage order.    */
void orc_mass_project(const double *phi, int nx, int ny, int nz, int walls_y, double target, double phi_min,
                      double phi_max, double *out)
{
    const int64_t n = (int64_t)nx * ny * nz;
    double sum_phi = 0.0, sum_w = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int y = (int)((i / nx) % ny);
        if (walls_y && (y == 0 || y == ny - 1)) continue;
        double q = (phi[i] - phi_min) / (phi_max - phi_min);
        q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
        sum_phi += phi[i];
        sum_w += 4.0 * q * (1.0 - q);
    }
    const double c = sum_w > 0.0 ? (target - sum_phi) / sum_w : 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int y = (int)((i / nx) % ny);
        if (walls_y && (y == 0 || y == ny - 1)) {
            out[i] = phi[i];
            continue;
        }
        double q = (phi[i] - phi_min) / (phi_max - phi_min);
        q = q < 0.0 ? 0.0 : (q > 1.0 ? 1.0 : q);
        out[i] = phi[i] + c * 4.0 * q * (1.0 - q);
    }
}
