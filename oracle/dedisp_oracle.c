/*
 * Oracle for brute-force incoherent de-dispersion -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation written from the paper
 * ("A GPU-based survey for millisecond radio transients using ARTEMIS",
 * Armour et al.).  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header,
 * table or constant with the GPU library and must never be reached from the
 * product path.
 *
 * Floating point is IEEE binary64 throughout; build with -ffp-contract=off so
 * that no multiply-add is fused (the order of operations below is the one the
 * shift table is defined by).
 */
#include <math.h>
#include <stdint.h>

/*
 * Shift table, section "Searching for radio transients".
 *
 * The cold-plasma dispersion law delays a channel at frequency f by a time
 * proportional to DM * f^-2.  Incoherent de-dispersion shifts every channel by
 * that delay, measured against the top of the band, before summing over
 * frequency.  The paper cites the law without writing it; the constant
 * 4148.808 s MHz^2 pc^-1 cm^3 and the form
 *     shift[c][d] = round(4148.808 * DM_d * (f_c^-2 - f_top^-2) / tsamp)
 * are the definition this code follows, evaluated as:
 *     f_c = f_top - c*df                      (channel 0 at f_top, descending)
 *     k_c = 4148.808 * (1/(f_c*f_c) - 1/(f_top*f_top)) / tsamp
 *     x   = DM_d * k_c
 *     shift = floor(x) + (x - floor(x) >= 0.5)   (round half up)
 * Output layout: shift[c * ndm + d] (channel-major).
 * Returns the largest entry, or -1 if any entry does not fit in int32.
 */
int64_t oracle_shift_table(int nchans, double f_top, double df, double tsamp,
                           const double *dm, int ndm, int32_t *shift)
{
    int64_t max_shift = 0;
    for (int c = 0; c < nchans; ++c) {
        double f = f_top - (double)c * df;
        double inv_f2 = 1.0 / (f * f);
        double inv_top2 = 1.0 / (f_top * f_top);
        double k = 4148.808 * (inv_f2 - inv_top2) / tsamp;
        for (int d = 0; d < ndm; ++d) {
            double x = dm[d] * k;
            double fl = floor(x);
            double frac = x - fl;
            double r = fl + (frac >= 0.5 ? 1.0 : 0.0);
            if (!(r >= 0.0) || r > 2147483647.0)
                return -1;
            shift[(int64_t)c * ndm + d] = (int32_t)r;
            if ((int64_t)r > max_shift)
                max_shift = (int64_t)r;
        }
    }
    return max_shift;
}

/*
 * De-dispersed time series, sections "Searching for radio transients" and
 * "Acceleration via GPU computing": for each requested trial DM d and output
 * sample t,
 *     out[d][t] = sum over c of in[c][t + shift[c][d]]
 * i.e. every channel is shifted by its delay for that trial and the channels
 * are then integrated over frequency.  Input row c starts at in + c*in_stride.
 *
 * rows[i] selects the trial DM written to out row i; the time range is
 * [t_begin, t_begin + t_count).  Channels are summed in ascending order, in
 * binary64 for floating input and in int64 for 8-bit input.
 */
void oracle_dedisperse_f32(const float *in, int64_t in_stride, int nchans,
                           const int32_t *shift, int ndm,
                           const int32_t *rows, int nrows,
                           int64_t t_begin, int64_t t_count, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nrows; ++i) {
        int d = rows[i];
        double *o = out + (int64_t)i * t_count;
        for (int64_t t = 0; t < t_count; ++t)
            o[t] = 0.0;
        for (int c = 0; c < nchans; ++c) {
            const float *src = in + (int64_t)c * in_stride + shift[(int64_t)c * ndm + d] + t_begin;
            for (int64_t t = 0; t < t_count; ++t)
                o[t] += (double)src[t];
        }
    }
}

void oracle_dedisperse_u8(const uint8_t *in, int64_t in_stride, int nchans,
                          const int32_t *shift, int ndm,
                          const int32_t *rows, int nrows,
                          int64_t t_begin, int64_t t_count, int64_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nrows; ++i) {
        int d = rows[i];
        int64_t *o = out + (int64_t)i * t_count;
        for (int64_t t = 0; t < t_count; ++t)
            o[t] = 0;
        for (int c = 0; c < nchans; ++c) {
            const uint8_t *src = in + (int64_t)c * in_stride + shift[(int64_t)c * ndm + d] + t_begin;
            for (int64_t t = 0; t < t_count; ++t)
                o[t] += (int64_t)src[t];
        }
    }
}

/* Number of OpenMP threads a parallel region of this library uses. */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
