/*
 * corr_oracle.h -- CPU FP64 oracle of the multiple-tau correlator.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library.
 */
#ifndef CORR_ORACLE_H
#define CORR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_corr oracle_corr;

/* n_ch independent channels, b = levels blocks of p = points values,
 * averaging factor m (2 <= m < p).  is_complex selects complex samples. */
oracle_corr *oracle_create(int64_t n_ch, int levels, int points, int m, int is_complex);
void oracle_destroy(oracle_corr *o);
/* One sample per channel (x_im only for complex correlators). */
int oracle_push(oracle_corr *o, const double *x_re, const double *x_im);
/* n_rows pushes of rows [n_rows][n_ch] (x_im likewise for complex records). */
int oracle_push_rows(oracle_corr *o, int64_t n_rows, const double *x_re, const double *x_im);
int64_t oracle_n_push(const oracle_corr *o);
/* Upper bound on the number of readout points: p + (b-1)(p - floor(p/m)). */
int oracle_max_out(const oracle_corr *o);
/* Group readout (mean over channels [ch_begin, ch_end)); lag times in
 * update steps (multiply by u*dt for physical time).  Returns n_out. */
int oracle_readout(const oracle_corr *o, int64_t ch_begin, int64_t ch_end, double *t_steps,
                   double *c_re, double *c_im, int64_t *count);
int oracle_readout_channel(const oracle_corr *o, int64_t ch, double *t_steps, double *c_re,
                           double *c_im, int64_t *count);
int oracle_raw(const oracle_corr *o, int64_t ch, double *sum_re, double *sum_im, int64_t *count);
double oracle_trapezoid(int n, const double *t, const double *c, double t_cut, double *running);
void oracle_rhok(const float *pos, int64_t n_atoms, const int32_t *kvec, int n_k, double box,
                 double *re, double *im);
int oracle_push_pair(oracle_corr *o, const double *x_re, const double *x_im, const double *y_re,
                     const double *y_im);
int oracle_currents(const float *pos, const float *vel, int64_t n_atoms, const int32_t *kvec,
                    int n_k, double box, double *re, double *im);
int oracle_partial_momentum(const double *vel, const int32_t *species, int64_t n_atoms,
                            const double *masses, int n_species, double volume, double *out);

#ifdef __cplusplus
}
#endif
#endif
