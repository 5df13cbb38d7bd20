/*
 * corr_oracle.c -- plain, slow, CPU reference of the on-the-fly multiple-tau
 * correlator (DL_POLY 5 paper, Section 2.2 "Correlation functions at runtime",
 * Appendix D, Algorithm 1 "Updating a correlator" and Algorithm 2 "Readout of
 * a correlation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or helper
 * with the GPU library, and the GPU library never calls it.
 *
 * Everything is double precision (complex double for complex observables).
 * A record correlates each channel with itself (oracle_push) or, in the pair
 * form of Algorithm 1, a first value x with a second value y
 * (oracle_push_pair): C(L) = <x(s) conj(y(s - L))>.
 * One independent correlator record per channel, updated recursively exactly
 * in the order Algorithm 1 gives (ring write, accumulate, cascade, lag loop,
 * cursor advance).  Where the printed algorithm is ambiguous the following
 * readings are taken (each is also listed with its justification in the
 * design notes of the repository):
 *   R1  the "valid shift" of a block is the number of values it has received,
 *       capped at p (a literal reading of the listing would reset it on wrap);
 *   R2  a block cascades when exactly m values have been accumulated, and the
 *       value passed down is their mean (sum in push order, divided by m);
 *   R3  the lag-0-inclusive branch is taken for the first block, not for the
 *       first cursor position;
 *   R4  the product is newest-sample times conj(lagged sample);
 *   R5  in blocks after the first, the lagged slot for lag L is (cursor - L)
 *       modulo p, i.e. the same lag convention as in the first block;
 *   R6  blocks after the first only accumulate lags L < (values received);
 *   R7/R8 readout walks block 0 over lags 0..p-1 and every later block over
 *       lags floor(p/m)..p-1, emitting each (block, lag) with a non-zero
 *       count; a channel's value is sum/count and a group value is the mean
 *       over channels of those per-channel values;
 *   R13 partially filled averaging accumulators are not flushed at readout;
 *   R14 Green-Kubo integrals use the trapezoid rule on the emitted lag grid,
 *       starting at t = 0, with linear interpolation of C inside the last
 *       interval when a cut-off falls between grid points.
 * The function that computes rho(k) follows the k-space density definition
 * of Section "Currents" (Eq. k-density): a direct sum of exp(i k.r) in double.
 * The currents function follows Eqs. long-current and trans-current of the
 * same section, with the readings
 *   R19 the bracket of Eq. trans-current closes after the projection:
 *       j_T = sum_i [v_i - (v_i . khat) khat] exp(i k.r_i);
 *   R20 the correlated channels of a k-vector are the longitudinal amplitude
 *       khat . j_L and the two transverse components e1 . j_T, e2 . j_T on a
 *       fixed orthonormal basis (khat, e1, e2): a = the Cartesian axis with
 *       the smallest |khat_a| (the first on ties), e1 = a - (a . khat) khat
 *       normalised, e2 = khat x e1.  C_L is the correlation of the first,
 *       C_T the mean of the other two (for k along z these are the paper's
 *       z, and x, y components).
 * The partial momentum density follows the mass-flux correction of Section
 * "Viscosity and thermal conductivity" (the equation for j_{I_s}), with the
 * reading
 *   R22 every atom of species s has the mass m_s; V = L^3; the output holds
 *       j_{I_s} for every species s, component alpha at 3 s + alpha.
 *
 * parity pins: see tests/test_oracle_*.py (brute-force Eq. (1) on block
 * averaged series, closed forms, invariants, hand-worked golden example).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "corr_oracle.h"

typedef double complex cplx;

struct oracle_corr {
    int64_t n_ch;
    int levels; /* b */
    int points; /* p */
    int m;
    int is_complex;
    int64_t n_push;
    /* per channel, per block: ring[p], sums[p], counts[p], cursor, filled,
     * accumulator, accumulated; plus blocks used.  Stored channel-major so
     * that each channel is an independent record, as in the paper. */
    cplx *ring;     /* [n_ch][b][p] */
    cplx *sums;     /* [n_ch][b][p] */
    int64_t *cnt;   /* [n_ch][b][p] */
    int *cursor;    /* [n_ch][b] */
    int *filled;    /* [n_ch][b] */
    cplx *acc;      /* [n_ch][b] */
    int *nacc;      /* [n_ch][b] */
    int *used;      /* [n_ch] */
    /* pair form (Algorithm 1 with x != y): ring and acc above hold y, these
     * hold x; allocated by the first oracle_push_pair */
    cplx *ringx;    /* [n_ch][b][p] */
    cplx *accx;     /* [n_ch][b] */
};

static size_t idx_bp(const oracle_corr *o, int64_t c, int k, int l)
{
    return ((size_t)c * (size_t)o->levels + (size_t)k) * (size_t)o->points + (size_t)l;
}

static size_t idx_b(const oracle_corr *o, int64_t c, int k)
{
    return (size_t)c * (size_t)o->levels + (size_t)k;
}

oracle_corr *oracle_create(int64_t n_ch, int levels, int points, int m, int is_complex)
{
    if (n_ch < 1 || levels < 1 || points < 2 || m < 2 || m >= points)
        return NULL;
    oracle_corr *o = (oracle_corr *)calloc(1, sizeof(*o));
    if (!o)
        return NULL;
    o->n_ch = n_ch;
    o->levels = levels;
    o->points = points;
    o->m = m;
    o->is_complex = is_complex ? 1 : 0;
    size_t nbp = (size_t)n_ch * (size_t)levels * (size_t)points;
    size_t nb = (size_t)n_ch * (size_t)levels;
    o->ring = (cplx *)calloc(nbp, sizeof(cplx));
    o->sums = (cplx *)calloc(nbp, sizeof(cplx));
    o->cnt = (int64_t *)calloc(nbp, sizeof(int64_t));
    o->cursor = (int *)calloc(nb, sizeof(int));
    o->filled = (int *)calloc(nb, sizeof(int));
    o->acc = (cplx *)calloc(nb, sizeof(cplx));
    o->nacc = (int *)calloc(nb, sizeof(int));
    o->used = (int *)calloc((size_t)n_ch, sizeof(int));
    if (!o->ring || !o->sums || !o->cnt || !o->cursor || !o->filled || !o->acc || !o->nacc ||
        !o->used) {
        oracle_destroy(o);
        return NULL;
    }
    return o;
}

void oracle_destroy(oracle_corr *o)
{
    if (!o)
        return;
    free(o->ring);
    free(o->sums);
    free(o->cnt);
    free(o->cursor);
    free(o->filled);
    free(o->acc);
    free(o->nacc);
    free(o->used);
    free(o->ringx);
    free(o->accx);
    free(o);
}

/* Algorithm 1, for one channel c, block k (0-based), new value v. */
static void update(oracle_corr *o, int64_t c, cplx v, int k)
{
    const int p = o->points;
    const int m = o->m;
    if (k >= o->levels) /* beyond the last block: nothing to do */
        return;
    if (o->used[c] < k + 1)
        o->used[c] = k + 1;

    size_t kb = idx_b(o, c, k);
    int cur = o->cursor[kb];
    o->ring[idx_bp(o, c, k, cur)] = v;
    if (o->filled[kb] < p) /* R1 */
        o->filled[kb] += 1;

    o->acc[kb] += v;
    o->nacc[kb] += 1;
    if (o->nacc[kb] == m) { /* R2 */
        cplx avg = o->acc[kb] / (double)m;
        update(o, c, avg, k + 1);
        o->acc[kb] = 0.0;
        o->nacc[kb] = 0;
    }

    /* R3-R6: lag loop of this block. */
    int lag0 = (k == 0) ? 0 : p / m;
    for (int L = lag0; L < p && L < o->filled[kb]; ++L) {
        int slot = ((cur - L) % p + p) % p;
        cplx r = o->ring[idx_bp(o, c, k, slot)];
        o->sums[idx_bp(o, c, k, L)] += v * conj(r); /* R4 */
        o->cnt[idx_bp(o, c, k, L)] += 1;
    }
    o->cursor[kb] = (cur + 1) % p;
}

/* Algorithm 1 with a pair of values: ring entry and block accumulator carry
 * (x, y), the block mean of both is passed down, and the lag product is the
 * newest x times conj(the lagged y) (R4), so C(L) = <x(s) conj(y(s - L))>. */
static void update_pair(oracle_corr *o, int64_t c, cplx x, cplx y, int k)
{
    const int p = o->points;
    const int m = o->m;
    if (k >= o->levels)
        return;
    if (o->used[c] < k + 1)
        o->used[c] = k + 1;

    size_t kb = idx_b(o, c, k);
    int cur = o->cursor[kb];
    o->ringx[idx_bp(o, c, k, cur)] = x;
    o->ring[idx_bp(o, c, k, cur)] = y;
    if (o->filled[kb] < p) /* R1 */
        o->filled[kb] += 1;

    o->accx[kb] += x;
    o->acc[kb] += y;
    o->nacc[kb] += 1;
    if (o->nacc[kb] == m) { /* R2 */
        cplx ax = o->accx[kb] / (double)m;
        cplx ay = o->acc[kb] / (double)m;
        update_pair(o, c, ax, ay, k + 1);
        o->accx[kb] = 0.0;
        o->acc[kb] = 0.0;
        o->nacc[kb] = 0;
    }

    int lag0 = (k == 0) ? 0 : p / m;
    for (int L = lag0; L < p && L < o->filled[kb]; ++L) {
        int slot = ((cur - L) % p + p) % p;
        cplx r = o->ring[idx_bp(o, c, k, slot)];
        o->sums[idx_bp(o, c, k, L)] += x * conj(r); /* R4 */
        o->cnt[idx_bp(o, c, k, L)] += 1;
    }
    o->cursor[kb] = (cur + 1) % p;
}

int oracle_push_pair(oracle_corr *o, const double *x_re, const double *x_im, const double *y_re,
                     const double *y_im)
{
    if (!o || !x_re || !y_re)
        return -1;
    if (o->is_complex && (!x_im || !y_im))
        return -1;
    if (!o->ringx) {
        if (o->n_push > 0) /* a record is either auto or pair from its first push */
            return -1;
        size_t nbp = (size_t)o->n_ch * (size_t)o->levels * (size_t)o->points;
        o->ringx = (cplx *)calloc(nbp, sizeof(cplx));
        o->accx = (cplx *)calloc((size_t)o->n_ch * (size_t)o->levels, sizeof(cplx));
        if (!o->ringx || !o->accx)
            return -1;
    }
    for (int64_t c = 0; c < o->n_ch; ++c) {
        cplx x = x_re[c], y = y_re[c];
        if (o->is_complex) {
            x = x_re[c] + x_im[c] * I;
            y = y_re[c] + y_im[c] * I;
        }
        update_pair(o, c, x, y, 0);
    }
    o->n_push += 1;
    return 0;
}

int oracle_push(oracle_corr *o, const double *x_re, const double *x_im)
{
    if (!o || !x_re)
        return -1;
    if (o->ringx) /* pair record */
        return -1;
    if (o->is_complex && !x_im)
        return -1;
    for (int64_t c = 0; c < o->n_ch; ++c) {
        cplx v = x_re[c];
        if (o->is_complex)
            v = x_re[c] + x_im[c] * I;
        update(o, c, v, 0);
    }
    o->n_push += 1;
    return 0;
}

/* n_rows consecutive pushes: row r is x_re + r * n_ch (and x_im likewise),
 * exactly n_rows calls of oracle_push in order. */
int oracle_push_rows(oracle_corr *o, int64_t n_rows, const double *x_re, const double *x_im)
{
    if (!o || n_rows < 0)
        return -1;
    for (int64_t r = 0; r < n_rows; ++r) {
        const int rc = oracle_push(o, x_re + r * o->n_ch, x_im ? x_im + r * o->n_ch : NULL);
        if (rc != 0)
            return rc;
    }
    return 0;
}

int64_t oracle_n_push(const oracle_corr *o) { return o ? o->n_push : -1; }

int oracle_max_out(const oracle_corr *o)
{
    if (!o)
        return -1;
    return o->points + (o->levels - 1) * (o->points - o->points / o->m);
}

/* Algorithm 2 for one channel: writes (level, lag, value, count) for every
 * (block, lag) with a non-zero count, in block-major, lag-minor order. */
static int readout_channel(const oracle_corr *o, int64_t c, int *lvl, int *lag, cplx *val,
                           int64_t *count)
{
    const int p = o->points;
    const int m = o->m;
    int n = 0;
    for (int k = 0; k < o->used[c]; ++k) { /* R7 */
        int lag0 = (k == 0) ? 0 : p / m;
        for (int L = lag0; L < p; ++L) {
            int64_t cn = o->cnt[idx_bp(o, c, k, L)];
            if (cn > 0) {
                lvl[n] = k;
                lag[n] = L;
                val[n] = o->sums[idx_bp(o, c, k, L)] / (double)cn; /* R8 */
                count[n] = cn;
                ++n;
            }
        }
    }
    return n;
}

static double lag_steps(int k, int L, int m)
{
    double t = (double)L;
    for (int i = 0; i < k; ++i)
        t *= (double)m;
    return t;
}

int oracle_readout(const oracle_corr *o, int64_t ch_begin, int64_t ch_end, double *t_steps,
                   double *c_re, double *c_im, int64_t *count)
{
    if (!o || ch_begin < 0 || ch_end > o->n_ch || ch_begin >= ch_end)
        return -1;
    int nmax = oracle_max_out(o);
    int *lvl = (int *)malloc(sizeof(int) * (size_t)nmax);
    int *lag = (int *)malloc(sizeof(int) * (size_t)nmax);
    cplx *val = (cplx *)malloc(sizeof(cplx) * (size_t)nmax);
    int64_t *cn = (int64_t *)malloc(sizeof(int64_t) * (size_t)nmax);
    cplx *mean = (cplx *)calloc((size_t)nmax, sizeof(cplx));
    if (!lvl || !lag || !val || !cn || !mean) {
        free(lvl); free(lag); free(val); free(cn); free(mean);
        return -2;
    }
    int n_out = -1;
    for (int64_t c = ch_begin; c < ch_end; ++c) {
        int n = readout_channel(o, c, lvl, lag, val, cn);
        if (n_out < 0) {
            n_out = n;
            for (int i = 0; i < n; ++i) {
                t_steps[i] = lag_steps(lvl[i], lag[i], o->m);
                count[i] = cn[i];
            }
        } else if (n != n_out) {
            n_out = -3; /* every channel of a group sees the same pushes */
            break;
        }
        for (int i = 0; i < n; ++i)
            mean[i] += val[i]; /* R8: values(tau) <- values(tau) + ... */
    }
    if (n_out > 0) {
        double inv = 1.0 / (double)(ch_end - ch_begin);
        for (int i = 0; i < n_out; ++i) {
            c_re[i] = creal(mean[i]) * inv;
            if (c_im)
                c_im[i] = cimag(mean[i]) * inv;
        }
    }
    free(lvl); free(lag); free(val); free(cn); free(mean);
    return n_out;
}

int oracle_readout_channel(const oracle_corr *o, int64_t ch, double *t_steps, double *c_re,
                           double *c_im, int64_t *count)
{
    return oracle_readout(o, ch, ch + 1, t_steps, c_re, c_im, count);
}

/* Raw per-(block, lag) state of one channel, for white-box checks:
 * sums and counts of block k, lag L at [k*p + L]. */
int oracle_raw(const oracle_corr *o, int64_t ch, double *sum_re, double *sum_im, int64_t *count)
{
    if (!o || ch < 0 || ch >= o->n_ch)
        return -1;
    size_t n = (size_t)o->levels * (size_t)o->points;
    for (size_t i = 0; i < n; ++i) {
        cplx s = o->sums[(size_t)ch * n + i];
        sum_re[i] = creal(s);
        if (sum_im)
            sum_im[i] = cimag(s);
        count[i] = o->cnt[(size_t)ch * n + i];
    }
    return 0;
}

/* Green-Kubo style running integral (R14): trapezoid rule over the points
 * (t_i, c_i) sorted by t, starting at t_0 (the lag-0 point).  running[i] is
 * the integral from t_0 to t_i.  Returns the integral up to t_cut, with c
 * linearly interpolated inside the interval containing t_cut; a cut-off past
 * the last point returns the full integral. */
double oracle_trapezoid(int n, const double *t, const double *c, double t_cut, double *running)
{
    if (n <= 0)
        return 0.0;
    double acc = 0.0;
    double at_cut = 0.0;
    int cut_done = 0;
    if (running)
        running[0] = 0.0;
    if (t_cut <= t[0]) {
        at_cut = 0.0;
        cut_done = 1;
    }
    for (int i = 1; i < n; ++i) {
        double dt = t[i] - t[i - 1];
        if (!cut_done && t_cut < t[i]) {
            double f = (t_cut - t[i - 1]) / dt;
            double c_cut = c[i - 1] + f * (c[i] - c[i - 1]);
            at_cut = acc + 0.5 * (t_cut - t[i - 1]) * (c[i - 1] + c_cut);
            cut_done = 1;
        }
        acc += 0.5 * dt * (c[i] + c[i - 1]);
        if (running)
            running[i] = acc;
    }
    if (!cut_done)
        at_cut = acc;
    return at_cut;
}

/* Eq. (k-density): n(k) = sum_j exp(i k . r_j), k = 2 pi n / L, for single
 * precision positions stored as three planes x[N], y[N], z[N]; evaluated
 * with double arguments, double sin/cos and a plain sequential sum. */
void oracle_rhok(const float *pos, int64_t n_atoms, const int32_t *kvec, int n_k, double box,
                 double *re, double *im)
{
    const float *x = pos;
    const float *y = pos + n_atoms;
    const float *z = pos + 2 * n_atoms;
    const double two_pi = 6.283185307179586476925286766559;
    for (int q = 0; q < n_k; ++q) {
        double kx = two_pi * (double)kvec[3 * q + 0] / box;
        double ky = two_pi * (double)kvec[3 * q + 1] / box;
        double kz = two_pi * (double)kvec[3 * q + 2] / box;
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n_atoms; ++j) {
            double ph = kx * (double)x[j] + ky * (double)y[j] + kz * (double)z[j];
            sr += cos(ph);
            si += sin(ph);
        }
        re[q] = sr;
        im[q] = si;
    }
}

/* Orthonormal basis (khat, e1, e2) of reading R20 for the integer vector n. */
static void current_basis(const int32_t *n, double khat[3], double e1[3], double e2[3])
{
    double len = sqrt((double)n[0] * n[0] + (double)n[1] * n[1] + (double)n[2] * n[2]);
    int a = 0;
    for (int d = 0; d < 3; ++d) {
        khat[d] = (double)n[d] / len;
    }
    for (int d = 1; d < 3; ++d)
        if (fabs(khat[d]) < fabs(khat[a])) a = d;
    double dot = khat[a];
    double nrm = 0.0;
    for (int d = 0; d < 3; ++d) {
        e1[d] = (d == a ? 1.0 : 0.0) - dot * khat[d];
        nrm += e1[d] * e1[d];
    }
    nrm = sqrt(nrm);
    for (int d = 0; d < 3; ++d) e1[d] /= nrm;
    e2[0] = khat[1] * e1[2] - khat[2] * e1[1];
    e2[1] = khat[2] * e1[0] - khat[0] * e1[2];
    e2[2] = khat[0] * e1[1] - khat[1] * e1[0];
}

/* Eqs. (long-current), (trans-current) with readings R19, R20: for every
 * k-vector q the complex current J = sum_j v_j exp(i k . r_j) (double
 * arguments, double sin/cos, sequential sums) and its components on the
 * basis (khat, e1, e2): out[3q] = khat . J, out[3q+1] = e1 . J,
 * out[3q+2] = e2 . J.  Positions and velocities are single precision planes
 * [3][N] each.  The zero vector has no direction and is not accepted
 * (returns -1); otherwise 0. */
int oracle_currents(const float *pos, const float *vel, int64_t n_atoms, const int32_t *kvec,
                    int n_k, double box, double *re, double *im)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int q = 0; q < n_k; ++q) {
        const int32_t *n = kvec + 3 * q;
        if (n[0] == 0 && n[1] == 0 && n[2] == 0) return -1;
        double k[3], khat[3], e1[3], e2[3];
        for (int d = 0; d < 3; ++d) k[d] = two_pi * (double)n[d] / box;
        current_basis(n, khat, e1, e2);
        double jr[3] = {0.0, 0.0, 0.0}, ji[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n_atoms; ++j) {
            double ph = 0.0;
            for (int d = 0; d < 3; ++d) ph += k[d] * (double)pos[d * n_atoms + j];
            const double c = cos(ph), s = sin(ph);
            for (int d = 0; d < 3; ++d) {
                jr[d] += (double)vel[d * n_atoms + j] * c;
                ji[d] += (double)vel[d * n_atoms + j] * s;
            }
        }
        const double *dirs[3] = {khat, e1, e2};
        for (int c = 0; c < 3; ++c) {
            double r = 0.0, i = 0.0;
            for (int d = 0; d < 3; ++d) {
                r += dirs[c][d] * jr[d];
                i += dirs[c][d] * ji[d];
            }
            re[3 * q + c] = r;
            im[3 * q + c] = i;
        }
    }
    return 0;
}

/* Partial momentum density of every species (Section "Viscosity and thermal
 * conductivity", the mass-flux correction; reading R22):
 * out[3 s + alpha] = (1/V) sum over atoms i with species[i] == s of
 * m_s v_alpha(i), one plain double sum per species and component in atom
 * order.  vel: [3][n_atoms]; species: [n_atoms] in [0, n_species).  Returns
 * -1 (output untouched) when a species id is out of range. */
int oracle_partial_momentum(const double *vel, const int32_t *species, int64_t n_atoms,
                            const double *masses, int n_species, double volume, double *out)
{
    for (int64_t i = 0; i < n_atoms; ++i)
        if (species[i] < 0 || species[i] >= n_species) return -1;
    for (int s = 0; s < n_species; ++s) {
        for (int d = 0; d < 3; ++d) {
            double sum = 0.0;
            for (int64_t i = 0; i < n_atoms; ++i)
                if (species[i] == s) sum += masses[s] * vel[d * n_atoms + i];
            out[3 * s + d] = sum / volume;
        }
    }
    return 0;
}
