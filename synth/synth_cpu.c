/*
 * synth_cpu.c -- seeded synthetic inputs (CPU side).
 *
 * These generators stand in for the molecular-dynamics observables the paper
 * correlates (atom velocities, global stress / heat-flux components and atom
 * positions for the k-space density).  They hold none of the correlator's
 * arithmetic.  synth_gpu.hip implements the same definitions on the GPU and
 * the two are bit-identical:
 *
 *  - random bits: the SplitMix64 output function (Steele, Lea & Flood,
 *    "Fast splittable pseudorandom number generators", OOPSLA 2014) applied
 *    to key + counter * gamma, i.e. element number `counter` of the
 *    SplitMix64 sequence seeded with `key`;  counter = (step << 32) |
 *    (channel << 2) | word, key = mix(seed * gamma + stream);
 *  - innovations: Irwin-Hall sum of twelve 20-bit midpoint uniforms minus 6,
 *    which is an exact single-precision number with mean 0 and variance
 *    1 - 2^-40;
 *  - Ornstein-Uhlenbeck recursion x_{t+1} = fma(a, x_t, round(b * xi)),
 *    x_0 = round(sigma * xi_0), with a and b supplied per channel group
 *    (computed once on the host in double and rounded).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SYNTH_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_key(uint64_t seed, uint64_t stream) { return mix64(seed * SYNTH_GAMMA + stream); }

uint64_t synth_bits(uint64_t key, uint64_t step, uint64_t channel, uint64_t word)
{
    uint64_t ctr = (step << 32) | (channel << 2) | word;
    return mix64(key + ctr * SYNTH_GAMMA);
}

/* Irwin-Hall innovation as an integer numerator n, xi = n * 2^-20. */
static inline int32_t xi_num(uint64_t key, uint64_t step, uint64_t channel)
{
    int32_t s = 0;
    for (uint64_t w = 0; w < 4; ++w) {
        uint64_t r = synth_bits(key, step, channel, w);
        s += (int32_t)(r & 0xFFFFF);
        s += (int32_t)((r >> 20) & 0xFFFFF);
        s += (int32_t)((r >> 40) & 0xFFFFF);
    }
    return s + 6 - 6 * (1 << 20);
}

float synth_xi_f32(uint64_t key, uint64_t step, uint64_t channel)
{
    return (float)xi_num(key, step, channel) * 0x1p-20f;
}

double synth_xi_f64(uint64_t key, uint64_t step, uint64_t channel)
{
    return (double)xi_num(key, step, channel) * 0x1p-20;
}

/*
 * OU series, single precision.  Channels: a list chan[n] of global channel
 * indices (or NULL meaning 0..n-1); the coefficient of channel c is
 * a[c / comps], b[c / comps] (comps channels share one coefficient pair,
 * e.g. the three velocity components of one atom).  state[n] holds x_{t-1}
 * on entry when t_begin > 0 and x_{t_begin + n_steps - 1} on exit.
 * out[s][n] receives x_{t_begin + s}.
 */
void synth_ou_f32(uint64_t key, int64_t n, const int64_t *chan, int comps, const float *a,
                  const float *b, float sigma, int64_t t_begin, int64_t n_steps, float *state,
                  float *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c = chan ? (uint64_t)chan[i] : (uint64_t)i;
        float ac = a[c / (uint64_t)comps];
        float bc = b[c / (uint64_t)comps];
        float x = state[i];
        for (int64_t s = 0; s < n_steps; ++s) {
            int64_t t = t_begin + s;
            float xi = synth_xi_f32(key, (uint64_t)t, c);
            if (t == 0)
                x = sigma * xi;
            else
                x = fmaf(ac, x, bc * xi);
            if (out)
                out[s * n + i] = x;
        }
        state[i] = x;
    }
}

void synth_ou_f64(uint64_t key, int64_t n, const int64_t *chan, int comps, const double *a,
                  const double *b, double sigma, int64_t t_begin, int64_t n_steps, double *state,
                  double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c = chan ? (uint64_t)chan[i] : (uint64_t)i;
        double ac = a[c / (uint64_t)comps];
        double bc = b[c / (uint64_t)comps];
        double x = state[i];
        for (int64_t s = 0; s < n_steps; ++s) {
            int64_t t = t_begin + s;
            double xi = synth_xi_f64(key, (uint64_t)t, c);
            if (t == 0)
                x = sigma * xi;
            else
                x = fma(ac, x, bc * xi);
            if (out)
                out[s * n + i] = x;
        }
        state[i] = x;
    }
}

/*
 * Positions r_j(t) = round(r0_j + d_j(t)) with d an OU displacement per
 * component (channel index of component q of atom j is q * n_atoms + j), all
 * single precision, stored as three planes [3][n_atoms] per step.
 */
void synth_positions(uint64_t key, int64_t n_atoms, const float *r0, float a_d, float b_d,
                     float sigma_d, int64_t t_begin, int64_t n_steps, float *d_state, float *out)
{
    for (int64_t c = 0; c < 3 * n_atoms; ++c) {
        float d = d_state[c];
        for (int64_t s = 0; s < n_steps; ++s) {
            int64_t t = t_begin + s;
            float xi = synth_xi_f32(key, (uint64_t)t, (uint64_t)c);
            if (t == 0)
                d = sigma_d * xi;
            else
                d = fmaf(a_d, d, b_d * xi);
            if (out)
                out[s * 3 * n_atoms + c] = r0[c] + d;
        }
        d_state[c] = d;
    }
}

/* Uniform double in [0,1) from 53 random bits of element `index`. */
void synth_uniform_f64(uint64_t key, int64_t n, uint64_t word, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)(synth_bits(key, 0, (uint64_t)i, word) >> 11) * 0x1p-53;
}
