/*
 * synth.c -- acquisition simulator for seeded synthetic RF data.
 *
 * Input generation only: it models the physics of the scan (point scatterers
 * echoing a Gaussian-windowed sinusoidal pulse back to the receivers).  It
 * contains no decoding and no beamforming; both the CPU oracle and the GPU
 * library only ever see the int16 data built from its output.
 *
 * Element response of decoded transmit i and receiver j:
 *   e_ij(t_n) = sum_s A_s * p(t_n - tof_ij(s)),   t_n = t0 + n / fs,
 *   p(t) = cos(2 pi fc t) * exp(-t^2 / (2 sigma^2)), sigma = 1 / (2 fc),
 * truncated at |t| <= 4 sigma.  The propagation model per mode:
 *   mode 0 (line elements, x-z plane): tof = (|s - tx|_xz + |s - rx|_xz) / c
 *   mode 1 (point receiver (x_i, y_j, 0)): tof = (tx(s) + |s - rx|) / c with
 *          tx = z_s (plane wave, focal = +inf) or the distance to the virtual
 *          source (xc, yc, focal < 0) minus |focal| (diverging wave)
 *   mode 2 (tilted plane wave theta_i from the columns, row receivers):
 *          tof = ((x_s - xc) sin theta_i + z_s cos theta_i + |s - row_j|_yz) / c
 *   mode 3 (virtual line source (x_i, focal) from the columns, row receivers):
 *          tof = (focal + sgn(z_s - focal) |s - src_i|_xz + |s - row_j|_yz) / c
 * Positions are in the array frame (metres); (xc, yc) is the array centre.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

void synth_echoes(int mode, int n_tx, int n_ch, int n_samples,
                  const double *tx_x,   /* n_tx: x of decoded transmit i            */
                  const double *rx_c,   /* n_ch: x (mode 0) or y (modes 1-3) of j   */
                  int n_scat, const double *sp, const double *amp,
                  double fs, double fc, double c, double t0,
                  double focal, const double *angles, double xc, double yc, double *e)
{
    const double sigma = 1.0 / (2.0 * fc);
    const double half = 4.0 * sigma;
    const double two_pi_fc = 2.0 * M_PI * fc;
    const double inv_2s2 = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(dynamic, 4)
    for (int ij = 0; ij < n_tx * n_ch; ++ij) {
        int i = ij / n_ch, j = ij % n_ch;
        double *trace = e + (size_t)ij * n_samples;
        for (int n = 0; n < n_samples; ++n) trace[n] = 0.0;
        for (int q = 0; q < n_scat; ++q) {
            double xs = sp[3 * q], ys = sp[3 * q + 1], zs = sp[3 * q + 2];
            double tof;
            if (mode == 0) {
                double dt = hypot(xs - tx_x[i], zs);
                double dr = hypot(xs - rx_c[j], zs);
                tof = (dt + dr) / c;
            } else if (mode == 1) {
                double dx = xs - tx_x[i], dy = ys - rx_c[j];
                double tx = zs;
                if (!isinf(focal))
                    tx = sqrt((xs - xc) * (xs - xc) + (ys - yc) * (ys - yc) +
                              (zs - focal) * (zs - focal)) - fabs(focal);
                tof = (tx + sqrt(dx * dx + dy * dy + zs * zs)) / c;
            } else {
                double tx;
                if (mode == 2) {
                    tx = (xs - xc) * sin(angles[i]) + zs * cos(angles[i]);
                } else {
                    double d = hypot(xs - tx_x[i], zs - focal);
                    tx = focal + (zs >= focal ? d : -d);
                }
                tof = (tx + hypot(ys - rx_c[j], zs)) / c;
            }
            long n_lo = (long)ceil((tof - half - t0) * fs);
            long n_hi = (long)floor((tof + half - t0) * fs);
            if (n_lo < 0) n_lo = 0;
            if (n_hi > n_samples - 1) n_hi = n_samples - 1;
            for (long n = n_lo; n <= n_hi; ++n) {
                double t = t0 + (double)n / fs - tof;
                trace[n] += amp[q] * cos(two_pi_fc * t) * exp(-t * t * inv_2s2);
            }
        }
    }
}
