/*
 * oracle.c -- plain FP64 CPU oracle for Hadamard aperture decoding and
 * delay-and-sum (DAS) beamforming.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: it recomputes every element
 * position, grid point, delay, interpolation weight and apodization weight
 * from the problem description, in double precision, with plain loops in the
 * order the paper states them.  No blocking, fusion or reordering.
 *
 * Paper: "An Open Source Realtime GPU Beamformer for RCA and TOBE Arrays"
 * (arXiv 2512.11086).  Where the paper is silent the reading used is stated at
 * the function.  Pins for every function live in tests/test_oracle_pins.py;
 * none of them re-types the formulas below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#include <omp.h>

/* ------------------------------------------------------------------------- */
/* Hadamard matrices and decoding (Sec. IV-A; Sec. VII-E)                     */
/* ------------------------------------------------------------------------- */

/* Sylvester construction, natural order: H[k][i] = (-1)^popcount(k & i).
 * Reading: the paper never names its Hadamard construction; the workloads use
 * Sylvester's.  Returns 0, or -1 if n is not a power of two. */
/* Worker threads of the OpenMP loops below (timing of the oracle on a given
 * number of host cores; no arithmetic).  n < 1 leaves the setting unchanged;
 * returns the count in effect. */
int oracle_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
}

int oracle_sylvester(int n, int8_t *H)
{
    if (n < 1 || (n & (n - 1)) != 0) return -1;
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < n; ++i) {
            int bits = k & i, parity = 0;
            while (bits) { parity ^= bits & 1; bits >>= 1; }
            H[(size_t)k * n + i] = parity ? -1 : 1;
        }
    return 0;
}

/* Decoding is a matrix product across the transmit axis (Sec. VII-E, first
 * paragraph; Sec. IV-A on FORCES/HERCULES resolving to an STA dataset).
 * Row k of H is the polarity pattern of transmit k, so the acquisition is
 * r[k] = sum_i H[k][i] e[i]; applying H^T gives N * e because H^T H = N I.
 * Reading: the output is left unscaled (N * e), in exact integers.
 *   e[i][j][t] = sum_k H[k][i] * r[k][j][t]                                  */
void oracle_decode(const int8_t *H, int n_tx, int n_ch, int n_samples,
                   const int16_t *r, int64_t *e)
{
    const size_t plane = (size_t)n_ch * n_samples;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n_tx; ++i)
        for (size_t jt = 0; jt < plane; ++jt) {
            int64_t acc = 0;
            for (int k = 0; k < n_tx; ++k)
                acc += (int64_t)H[(size_t)k * n_tx + i] * (int64_t)r[(size_t)k * plane + jt];
            e[(size_t)i * plane + jt] = acc;
        }
}

/* ------------------------------------------------------------------------- */
/* Window, interpolation (Eq. 3; Sec. IV-B)                                   */
/* ------------------------------------------------------------------------- */

/* Hann window, Eq. 3: cos^2(pi u) for |u| < 1/2, else 0. */
double oracle_hann(double u)
{
    if (fabs(u) < 0.5) {
        double cu = cos(M_PI * u);
        return cu * cu;
    }
    return 0.0;
}

/* Sample n of a trace; zero outside [0, S).  Reading: the paper zero-pads the
 * signal ends (Sec. VII-D, LDS filtering paragraph). */
static double tap(const double *trace, int S, long n)
{
    return (n >= 0 && n < S) ? trace[n] : 0.0;
}

/* Fractional-delay read of a trace at sample position s (Sec. IV-B; Table I
 * lists nearest, linear and cubic Hermite).  Reading for "4-point cubic
 * hermite": Catmull-Rom tangents (p[n+1] - p[n-1]) / 2, written as the cubic
 * Hermite basis h00..h11 with those tangents, so the curve has a continuous
 * derivative as the paper requires.
 *   n = floor(s), t = s - n, p_k = e[n+k], k = -1..2.                        */
double oracle_interp(const double *trace, int S, double s, int mode)
{
    if (mode == ORACLE_NEAREST)
        return tap(trace, S, (long)floor(s + 0.5));
    long n = (long)floor(s);
    double t = s - (double)n;
    double p0 = tap(trace, S, n), p1 = tap(trace, S, n + 1);
    if (mode == ORACLE_LINEAR)
        return (1.0 - t) * p0 + t * p1;
    double pm = tap(trace, S, n - 1), p2 = tap(trace, S, n + 2);
    double m0 = 0.5 * (p1 - pm), m1 = 0.5 * (p2 - p0);     /* tangents */
    double t2 = t * t, t3 = t2 * t;
    double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t;
    double h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    return h00 * p0 + h10 * m0 + h01 * p1 + h11 * m1;
}

/* d/ds of oracle_interp (zero almost everywhere for nearest). */
double oracle_interp_deriv(const double *trace, int S, double s, int mode)
{
    if (mode == ORACLE_NEAREST) return 0.0;
    long n = (long)floor(s);
    double t = s - (double)n;
    double p0 = tap(trace, S, n), p1 = tap(trace, S, n + 1);
    if (mode == ORACLE_LINEAR) return p1 - p0;
    double pm = tap(trace, S, n - 1), p2 = tap(trace, S, n + 2);
    double m0 = 0.5 * (p1 - pm), m1 = 0.5 * (p2 - p0);
    double t2 = t * t;
    double d00 = 6 * t2 - 6 * t, d10 = 3 * t2 - 4 * t + 1;
    double d01 = -6 * t2 + 6 * t, d11 = 3 * t2 - 2 * t;
    return d00 * p0 + d10 * m0 + d01 * p1 + d11 * m1;
}

/* Weights w_k(t), k = -1..2, of the same interpolator: v = sum_k w_k p_k.
 * Used by the adjoint (the transpose of the read). */
static void interp_weights(double t, int mode, double w[4])
{
    w[0] = w[1] = w[2] = w[3] = 0.0;
    if (mode == ORACLE_LINEAR) { w[1] = 1.0 - t; w[2] = t; return; }
    double t2 = t * t, t3 = t2 * t;
    double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t;
    double h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    /* v = h00 p0 + h10 (p1 - pm)/2 + h01 p1 + h11 (p2 - p0)/2 */
    w[0] = -0.5 * h10;
    w[1] = h00 - 0.5 * h11;
    w[2] = h01 + 0.5 * h10;
    w[3] = 0.5 * h11;
}

/* ------------------------------------------------------------------------- */
/* Geometry (Sec. VI-B, data description; Fig. das_dispatch)                  */
/* ------------------------------------------------------------------------- */

/* Grid point of output index (ix, iy, iz): inclusive linspace between the
 * region bounds on each axis (a single point when the axis has one sample),
 * in the global frame, then mapped to the array frame by the 4x4 affine of
 * the data description (row-major, last row 0 0 0 1).  The array frame has its
 * origin at the centre of the corner element and z along the array normal. */
static void voxel_position(const oracle_geom *g, int ix, int iy, int iz, double p[3])
{
    int idx[3] = {ix, iy, iz};
    double q[3];
    for (int a = 0; a < 3; ++a) {
        int N = g->dims[a];
        q[a] = (N > 1) ? g->gmin[a] + idx[a] * (g->gmax[a] - g->gmin[a]) / (double)(N - 1)
                       : g->gmin[a];
    }
    for (int r = 0; r < 3; ++r)
        p[r] = g->xdc[4 * r + 0] * q[0] + g->xdc[4 * r + 1] * q[1] + g->xdc[4 * r + 2] * q[2] +
               g->xdc[4 * r + 3];
}

/* Element positions in the array frame.  Element column c sits at
 * x = c * pitch_x, row r at y = r * pitch_y, z = 0.
 * FORCES: decoded index i is the transmit column tx_elements[i]; data channel
 *   j is the receive column channel_map[j] (both line elements along y).
 * HERCULES: decoded index i is column tx_elements[i] and channel j is row
 *   channel_map[j]; the pair (i, j) is one element of the recovered 2D
 *   receive aperture (Sec. IV-A). */
static double elem_x(const oracle_geom *g, int i) { return g->tx_elements[i] * g->pitch[0]; }
static double chan_coord(const oracle_geom *g, int j)
{
    return g->mode == ORACLE_FORCES ? g->channel_map[j] * g->pitch[0]
                                    : g->channel_map[j] * g->pitch[1];
}
/* Centre of the element grid in the array frame. */
static double centre_x(const oracle_geom *g) { return 0.5 * (g->n_elem[0] - 1) * g->pitch[0]; }
static double centre_y(const oracle_geom *g) { return 0.5 * (g->n_elem[1] - 1) * g->pitch[1]; }

/* Round-trip time of flight and receive apodization of one (point, i, j).
 * FORCES (Eq. 1 with the decoded STA dataset): the transmit is a cylindrical
 *   wave from column x_i and the receive is column x_j, both in the x-z plane:
 *   tof = (sqrt((x-x_i)^2 + z^2) + sqrt((x-x_j)^2 + z^2)) / c.
 * HERCULES: plane-wave transmit along the array normal (tof_tx = z / c) and a
 *   point receiver at (x_i, y_j, 0): tof = (z + |p - (x_i, y_j, 0)|) / c.
 * Apodization (Eqs. 2-3), receive only (transmit apodization is 1 for
 *   unfocused transmits):  a = W(F# * rho / z), rho = lateral distance from
 *   the receiver (|x - x_j| for FORCES, radial for HERCULES, |y - y_j| for the
 *   row receivers of TPW and VLS).
 * Reading: points with z <= 0 (on or behind the array) get a = 0; F# = 0
 *   disables apodization (a = 1). */
static void tof_apod(const oracle_geom *g, const double p[3], int i, int j,
                     double *tof, double *apod)
{
    double x = p[0], y = p[1], z = p[2];
    double rho;
    if (g->mode == ORACLE_FORCES) {
        double xt = elem_x(g, i), xr = chan_coord(g, j);
        double dt = sqrt((x - xt) * (x - xt) + z * z);
        double dr = sqrt((x - xr) * (x - xr) + z * z);
        *tof = (dt + dr) / g->c;
        rho = fabs(x - xr);
    } else if (g->mode == ORACLE_HERCULES) {
        double xe = elem_x(g, i), ye = chan_coord(g, j);
        double rho2 = (x - xe) * (x - xe) + (y - ye) * (y - ye);
        /* transmit: plane wave (z), or a diverging wave from the virtual point
         * source v = (centre, focal_depth < 0) that crosses the array centre at
         * t = 0: |p - v| - |focal_depth| */
        double tx = z;
        if (!isinf(g->focal_depth)) {
            double dx = x - centre_x(g), dy = y - centre_y(g), dz = z - g->focal_depth;
            tx = sqrt(dx * dx + dy * dy + dz * dz) + g->focal_depth;
        }
        *tof = (tx + sqrt(rho2 + z * z)) / g->c;
        rho = sqrt(rho2);
    } else {
        /* Row-column volumes: columns transmit, rows (line elements along x at
         * y_j) receive a cylindrical wave in the y-z plane.
         * TPW: plane wave tilted by theta_i in the x-z plane, crossing the
         *      array centre at t = 0: (x - x_c) sin(theta) + z cos(theta).
         * VLS: cylindrical wave through the virtual line source (x_i, z_f),
         *      zero delay at the element: z_f + sgn(z - z_f) |(x, z) - (x_i, z_f)|
         *      (z_f > 0 focused, z_f < 0 diverging; sgn(0) = +1). */
        double ye = chan_coord(g, j);
        double tx;
        if (g->mode == ORACLE_TPW) {
            double th = g->tx_angles[i];
            tx = (x - centre_x(g)) * sin(th) + z * cos(th);
        } else {
            double xi = elem_x(g, i), zf = g->focal_depth;
            double d = sqrt((x - xi) * (x - xi) + (z - zf) * (z - zf));
            tx = zf + (z - zf >= 0.0 ? d : -d);
        }
        *tof = (tx + sqrt((y - ye) * (y - ye) + z * z)) / g->c;
        rho = fabs(y - ye);
    }
    if (z <= 0.0) { *apod = 0.0; return; }
    *apod = (g->f_number == 0.0) ? 1.0 : oracle_hann(g->f_number * rho / z);
}

/* Sample position of a time of flight: s = (tof - t0) * fs. */
static double sample_pos(const oracle_geom *g, double tof) { return (tof - g->t0) * g->fs; }

/* Eq. 1: HR(p) = sum_i a_tx sum_j a_rx(p) r_ij(tof_ij(p)), with a_tx = 1. */
static double das_point(const oracle_geom *g, const double *e, int64_t v)
{
    int Nx = g->dims[0], Nz = g->dims[2];
    int iz = (int)(v % Nz), ix = (int)((v / Nz) % Nx), iy = (int)(v / ((int64_t)Nz * Nx));
    double p[3];
    voxel_position(g, ix, iy, iz, p);
    double acc = 0.0;
    for (int i = 0; i < g->n_tx; ++i)
        for (int j = 0; j < g->n_ch; ++j) {
            double tof, a;
            tof_apod(g, p, i, j, &tof, &a);
            if (a == 0.0) continue;
            const double *trace = e + ((size_t)i * g->n_ch + j) * g->n_samples;
            acc += a * oracle_interp(trace, g->n_samples, sample_pos(g, tof), g->interp);
        }
    return acc;
}

static int64_t n_voxels(const oracle_geom *g)
{
    return (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
}

/* Full image, layout out[iy][ix][iz] (z fastest). */
void oracle_das(const oracle_geom *g, const double *e, double *out)
{
    int64_t nv = n_voxels(g);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < nv; ++v) out[v] = das_point(g, e, v);
}

/* Listed voxels only (linear indices into the same layout). */
void oracle_das_points(const oracle_geom *g, const double *e, const int64_t *vox, int64_t n,
                       double *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n; ++q) out[q] = das_point(g, e, vox[q]);
}

/* ------------------------------------------------------------------------- */
/* Adjoint of DAS and the sound-speed derivative                              */
/* ------------------------------------------------------------------------- */

/* Transpose of the linear map e -> HR for a fixed sound speed:
 *   grad_e[i][j][n+k] += G(p) * a(p,i,j) * w_k(t(p,i,j)).
 * Parallel over traces (i, j); every trace loops over all voxels. */
void oracle_das_adjoint_e(const oracle_geom *g, const double *G, double *grad_e)
{
    const int S = g->n_samples;
    const int64_t nv = n_voxels(g);
    const int Nx = g->dims[0], Nz = g->dims[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int ij = 0; ij < g->n_tx * g->n_ch; ++ij) {
        int i = ij / g->n_ch, j = ij % g->n_ch;
        double *ge = grad_e + (size_t)ij * S;
        for (int n = 0; n < S; ++n) ge[n] = 0.0;
        for (int64_t v = 0; v < nv; ++v) {
            if (G[v] == 0.0) continue;
            int iz = (int)(v % Nz), ix = (int)((v / Nz) % Nx), iy = (int)(v / ((int64_t)Nz * Nx));
            double p[3], tof, a;
            voxel_position(g, ix, iy, iz, p);
            tof_apod(g, p, i, j, &tof, &a);
            if (a == 0.0) continue;
            double s = sample_pos(g, tof);
            if (g->interp == ORACLE_NEAREST) {
                long n = (long)floor(s + 0.5);
                if (n >= 0 && n < S) ge[n] += G[v] * a;
                continue;
            }
            long n = (long)floor(s);
            double w[4];
            interp_weights(s - (double)n, g->interp, w);
            for (int k = -1; k <= 2; ++k) {
                long m = n + k;
                if (m >= 0 && m < S) ge[m] += G[v] * a * w[k + 1];
            }
        }
    }
}

/* Per-voxel derivative of HR with respect to the sound speed c.  Only the
 * delay depends on c (the apodization does not):
 *   s = (tof(c) - t0) fs, tof = path / c  =>  ds/dc = -tof fs / c
 *   dHR/dc = sum_ij a * v'(s) * ds/dc. */
void oracle_das_dc(const oracle_geom *g, const double *e, double *dout)
{
    const int64_t nv = n_voxels(g);
    const int Nx = g->dims[0], Nz = g->dims[2];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < nv; ++v) {
        int iz = (int)(v % Nz), ix = (int)((v / Nz) % Nx), iy = (int)(v / ((int64_t)Nz * Nx));
        double p[3];
        voxel_position(g, ix, iy, iz, p);
        double acc = 0.0;
        for (int i = 0; i < g->n_tx; ++i)
            for (int j = 0; j < g->n_ch; ++j) {
                double tof, a;
                tof_apod(g, p, i, j, &tof, &a);
                if (a == 0.0) continue;
                const double *trace = e + ((size_t)i * g->n_ch + j) * g->n_samples;
                double ds_dc = -tof * g->fs / g->c;
                acc += a * oracle_interp_deriv(trace, g->n_samples, sample_pos(g, tof), g->interp) *
                       ds_dc;
            }
        dout[v] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* Image-sharpness loss                                                      */
/* ------------------------------------------------------------------------- */

/* Negative normalised L4 norm of one image.  Reading: L = -sum I^4 / (sum I^2)^2
 * (a monotone transform of -||I||_4 / ||I||_2 with the same stationary points).
 * grad (nullable) receives dL/dI = -4 I^3 / Q^2 + 4 I P / Q^3, P = sum I^4,
 * Q = sum I^2.  An all-zero image gives L = 0 and a zero gradient. */
double oracle_sharpness(const double *img, int64_t n, double *grad)
{
    double P = 0.0, Q = 0.0;
    for (int64_t q = 0; q < n; ++q) {
        double x2 = img[q] * img[q];
        Q += x2;
        P += x2 * x2;
    }
    if (Q == 0.0) {
        if (grad) for (int64_t q = 0; q < n; ++q) grad[q] = 0.0;
        return 0.0;
    }
    if (grad)
        for (int64_t q = 0; q < n; ++q) {
            double x = img[q];
            grad[q] = -4.0 * x * x * x / (Q * Q) + 4.0 * x * P / (Q * Q * Q);
        }
    return -P / (Q * Q);
}

/* ------------------------------------------------------------------------- */
/* Demodulation, filtering, decimation (Eq. 4; Sec. VII-D; Sec. VII-C order)  */
/* ------------------------------------------------------------------------- */

/* Eq. 4, IQ[n] = LPF{ s[n] exp(-j 2 pi fd n / fs) }, in the paper's order:
 * first every input sample is mixed with the complex exponential at its own
 * index, then the FIR filter h (the baseband matched filter or a plain
 * low-pass; real or complex taps) is applied as a convolution, then every
 * D-th filter output is kept (decimation comes after the low-pass, which
 * must precede it):
 *   m[n]  = x[n] (cos(2 pi r n) - j sin(2 pi r n)),    r = fd / fs
 *   y[n]  = sum_{k=0}^{N_f-1} h[k] m[n-k],             m[n < 0] = 0
 *   IQ[q] = y[q D],                                    q = 0 .. ceil(S / D) - 1
 * Readings: n counts from sample 0 of the record; the convolution is causal
 * with the signal start zero-padded (the paper pads the start with zeros in
 * its LDS filter); no group-delay compensation (a caller folds the filter
 * delay into t0); output q is the filter output at input sample q D.
 * x: [n_traces][S] int16; y: [n_traces][n_out][2] (re, im), double. */
void oracle_demod(const int16_t *x, int n_traces, int S, const double *h_re, const double *h_im,
                  int n_taps, double fd_over_fs, int D, double *y)
{
    const int n_out = (S + D - 1) / D;
#pragma omp parallel
    {
        double *mr = malloc(sizeof(double) * (size_t)S);
        double *mi = malloc(sizeof(double) * (size_t)S);
#pragma omp for schedule(static)
        for (int tr = 0; tr < n_traces; ++tr) {
            const int16_t *xs = x + (size_t)tr * S;
            for (int n = 0; n < S; ++n) {
                double ph = 2.0 * M_PI * fd_over_fs * (double)n;
                mr[n] = (double)xs[n] * cos(ph);
                mi[n] = -(double)xs[n] * sin(ph);
            }
            double *yo = y + (size_t)tr * n_out * 2;
            for (int q = 0; q < n_out; ++q) {
                const long n = (long)q * D;
                double ar = 0.0, ai = 0.0;
                for (int k = 0; k < n_taps; ++k) {
                    long idx = n - k;
                    if (idx < 0) break;
                    double hr = h_re[k], hi = h_im ? h_im[k] : 0.0;
                    ar += hr * mr[idx] - hi * mi[idx];
                    ai += hr * mi[idx] + hi * mr[idx];
                }
                yo[2 * q] = ar;
                yo[2 * q + 1] = ai;
            }
        }
        free(mr);
        free(mi);
    }
}

/* Conversion of the filtered result back to 16-bit integers (Sec. VII-C:
 * filter gains <= 1 keep the data in 16 bits).  Reading: round to nearest
 * with ties to even, saturating at the int16 limits. */
void oracle_quantise_i16(const double *y, int64_t n, int16_t *q)
{
    for (int64_t i = 0; i < n; ++i) {
        double r = nearbyint(y[i]);
        if (r > 32767.0) r = 32767.0;
        if (r < -32768.0) r = -32768.0;
        q[i] = (int16_t)r;
    }
}

/* ------------------------------------------------------------------------- */
/* IQ (complex baseband) beamforming                                          */
/* ------------------------------------------------------------------------- */

/* Eq. 1 on demodulated data: each term reads the complex trace at the sample
 * position s = (tof - t0) fs (fs is the IQ sampling rate) with the same
 * interpolator applied to the real and imaginary parts, then restores the
 * carrier phase that the mix of Eq. 4 removed at that record time:
 *   HR(p) = sum_ij a(p,i,j) IQ_ij(s) exp(+j 2 pi fd (tof - t0)).
 * Reading: the phase restored is that of the record time tof - t0 (the mix
 * counts n from sample 0, whose time is t0), so the terms of a scatterer add
 * coherently across traces. */
static void das_point_iq(const oracle_geom *g, double fd, const double *er, const double *ei,
                         int64_t v, double *out_re, double *out_im)
{
    int Nx = g->dims[0], Nz = g->dims[2];
    int iz = (int)(v % Nz), ix = (int)((v / Nz) % Nx), iy = (int)(v / ((int64_t)Nz * Nx));
    double p[3];
    voxel_position(g, ix, iy, iz, p);
    double acc_r = 0.0, acc_i = 0.0;
    for (int i = 0; i < g->n_tx; ++i)
        for (int j = 0; j < g->n_ch; ++j) {
            double tof, a;
            tof_apod(g, p, i, j, &tof, &a);
            if (a == 0.0) continue;
            size_t off = ((size_t)i * g->n_ch + j) * g->n_samples;
            double s = sample_pos(g, tof);
            double vr = oracle_interp(er + off, g->n_samples, s, g->interp);
            double vi = oracle_interp(ei + off, g->n_samples, s, g->interp);
            double ph = 2.0 * M_PI * fd * (tof - g->t0);
            double c = cos(ph), sn = sin(ph);
            acc_r += a * (vr * c - vi * sn);
            acc_i += a * (vr * sn + vi * c);
        }
    *out_re = acc_r;
    *out_im = acc_i;
}

/* Full complex image: out_re / out_im [iy][ix][iz]; e_re / e_im are the real
 * and imaginary planes of the decoded data [n_tx][n_ch][n_samples]. */
void oracle_das_iq(const oracle_geom *g, double fd, const double *e_re, const double *e_im,
                   double *out_re, double *out_im)
{
    int64_t nv = n_voxels(g);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < nv; ++v) das_point_iq(g, fd, e_re, e_im, v, &out_re[v], &out_im[v]);
}

void oracle_das_iq_points(const oracle_geom *g, double fd, const double *e_re, const double *e_im,
                          const int64_t *vox, int64_t n, double *out_re, double *out_im)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n; ++q)
        das_point_iq(g, fd, e_re, e_im, vox[q], &out_re[q], &out_im[q]);
}

/* ------------------------------------------------------------------------- */
/* Envelope and display compression (the stage after DAS)                     */
/* ------------------------------------------------------------------------- */

/* Envelope of an RF image along the depth axis through the analytic signal
 * (the paper runs a Hilbert transform after beamforming), by the discrete
 * Fourier definition, one depth column at a time:
 *   X[k]   = sum_n x[n] exp(-j 2 pi k n / N)
 *   Xa[k]  = h[k] X[k],  h = 1 at k = 0 and (N even) k = N/2, 2 for
 *            0 < k < N/2, 0 for the negative frequencies
 *   xa[n]  = (1/N) sum_k Xa[k] exp(+j 2 pi k n / N)
 *   env[n] = |xa[n]|
 * Reading: the transform is circular over the N depth samples of a column
 * (an FFT of the column's own length, no padding).  img and env:
 * [n_cols][N], depth fastest.  Plain O(N^2) sums in FP64. */
void oracle_envelope(const double *img, int64_t n_cols, int N, double *env)
{
#pragma omp parallel
    {
        double *Xr = malloc(sizeof(double) * (size_t)N);
        double *Xi = malloc(sizeof(double) * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t col = 0; col < n_cols; ++col) {
            const double *x = img + (size_t)col * N;
            for (int k = 0; k < N; ++k) {
                double ar = 0.0, ai = 0.0;
                for (int n = 0; n < N; ++n) {
                    double ph = -2.0 * M_PI * (double)(((long)k * n) % N) / N;
                    ar += x[n] * cos(ph);
                    ai += x[n] * sin(ph);
                }
                double h = (k == 0 || 2 * k == N) ? 1.0 : (2 * k < N ? 2.0 : 0.0);
                Xr[k] = h * ar;
                Xi[k] = h * ai;
            }
            for (int n = 0; n < N; ++n) {
                double ar = 0.0, ai = 0.0;
                for (int k = 0; k < N; ++k) {
                    double ph = 2.0 * M_PI * (double)(((long)k * n) % N) / N;
                    double c = cos(ph), s = sin(ph);
                    ar += Xr[k] * c - Xi[k] * s;
                    ai += Xr[k] * s + Xi[k] * c;
                }
                env[(size_t)col * N + n] = sqrt(ar * ar + ai * ai) / N;
            }
        }
        free(Xr);
        free(Xi);
    }
}

/* Display compression of an envelope (the paper's live view shows a log scale
 * with an adjustable dynamic range or a power scale with an adjustable
 * threshold).  Readings:
 *   mode 0 (none):  y = env
 *   mode 1 (log):   y = max(20 log10(env / ref), -param)   (param = dynamic range, dB)
 *   mode 2 (power): y = min(env / ref, 1)^param             (ref = threshold, param = exponent)
 * ref <= 0 takes the maximum of env over the n values; an all-zero envelope
 * then gives -param (log) or 0 (power). */
void oracle_compress(const double *env, int64_t n, int mode, double ref, double param,
                     double *out)
{
    if (ref <= 0.0) {
        ref = 0.0;
        for (int64_t i = 0; i < n; ++i)
            if (env[i] > ref) ref = env[i];
    }
    for (int64_t i = 0; i < n; ++i) {
        double v = env[i];
        if (mode == 1) {
            double db = (ref > 0.0 && v > 0.0) ? 20.0 * log10(v / ref) : -INFINITY;
            out[i] = db > -param ? db : -param;
        } else if (mode == 2) {
            double r = ref > 0.0 ? v / ref : 0.0;
            out[i] = pow(r < 1.0 ? r : 1.0, param);
        } else {
            out[i] = v;
        }
    }
}
