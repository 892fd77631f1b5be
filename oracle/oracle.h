/*
 * oracle.h -- declarations of the FP64 CPU oracle (test infrastructure only;
 * see oracle.c).  Not included by, and shares nothing with, the GPU library.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

enum { ORACLE_FORCES = 0, ORACLE_HERCULES = 1, ORACLE_TPW = 2, ORACLE_VLS = 3 };
enum { ORACLE_NEAREST = 0, ORACLE_LINEAR = 1, ORACLE_CUBIC = 2 };

typedef struct {
    int mode;                  /* ORACLE_FORCES (2D) or ORACLE_HERCULES (3D)        */
    int n_tx, n_ch, n_samples; /* decoded transmits, data channels, samples        */
    const int32_t *tx_elements;/* n_tx: element column of decoded index i         */
    const int32_t *channel_map;/* n_ch: element column (FORCES) / row (HERCULES)  */
    double pitch[2];           /* column pitch (x), row pitch (y), metres          */
    double xdc[16];            /* row-major 4x4 affine, global -> array frame      */
    double fs, c, t0;          /* Hz, m/s, s (time of sample 0)                    */
    double f_number;           /* receive F#; 0 disables apodization               */
    int interp;                /* ORACLE_NEAREST / ORACLE_LINEAR / ORACLE_CUBIC    */
    int dims[3];               /* Nx, Ny, Nz                                       */
    double gmin[3], gmax[3];   /* inclusive region bounds, global frame, metres    */
    int n_elem[2];             /* element columns, rows (array centre for TPW and  */
                               /* the diverging HERCULES source)                   */
    double focal_depth;        /* HERCULES: +inf plane wave, < 0 diverging source; */
                               /* VLS: depth of the virtual line sources (!= 0)    */
    const double *tx_angles;   /* TPW: n_tx tilt angles, radians                   */
} oracle_geom;

int oracle_threads(int n);
int oracle_sylvester(int n, int8_t *H);
void oracle_decode(const int8_t *H, int n_tx, int n_ch, int n_samples, const int16_t *r,
                   int64_t *e);
double oracle_hann(double u);
double oracle_interp(const double *trace, int S, double s, int mode);
double oracle_interp_deriv(const double *trace, int S, double s, int mode);
void oracle_das(const oracle_geom *g, const double *e, double *out);
void oracle_das_points(const oracle_geom *g, const double *e, const int64_t *vox, int64_t n,
                       double *out);
void oracle_das_adjoint_e(const oracle_geom *g, const double *G, double *grad_e);
void oracle_das_dc(const oracle_geom *g, const double *e, double *dout);
double oracle_sharpness(const double *img, int64_t n, double *grad);
void oracle_demod(const int16_t *x, int n_traces, int S, const double *h_re, const double *h_im,
                  int n_taps, double fd_over_fs, int D, double *y);
void oracle_quantise_i16(const double *y, int64_t n, int16_t *q);
void oracle_das_iq(const oracle_geom *g, double fd, const double *e_re, const double *e_im,
                   double *out_re, double *out_im);
void oracle_envelope(const double *img, int64_t n_cols, int N, double *env);
void oracle_compress(const double *env, int64_t n, int mode, double ref, double param,
                     double *out);
void oracle_das_iq_points(const oracle_geom *g, double fd, const double *e_re, const double *e_im,
                          const int64_t *vox, int64_t n, double *out_re, double *out_im);

#endif
