/*
 * Plain CPU oracle for the AARTFAAC FX-correlator hot path (arXiv 1609.04205).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It is written from the paper's description, in double
 * precision (and exact 64-bit integers for the int8 path), as direct sums
 * with no FFT, no blocking and no reordering beyond the definitions below.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 *
 * Definitions followed (P channels, T taps, h the prototype filter taps in
 * the order h[t*P + p]):
 *   channeliser  (Sec. "Polyphase Filterbank": a bank of T-tap FIR filters,
 *                one per branch, followed by a P-point complex FFT)
 *       u[s][p] = sum_{t<T} h[t*P+p] * x[(s+t)*P + p]
 *       y[s][k] = sum_{p<P} u[s][p] * exp(-2 pi i k p / P)
 *   requantiser  (Sec. "LOFAR Digital Processing", bit modes trade bits for
 *                dynamic range): q = clamp(rint(y * gain), -127, 127) of
 *                float32 y and gain, the exact product rounded once to an
 *                integer, ties to even
 *   correlator   (Sec. "Correlation Kernel": per channel, the covariance of
 *                every pair of receivers integrated over time, one triangle
 *                of the Hermitian matrix)
 *       V[i][j] = sum_s z_i(s) * conj(z_j(s)),  for antennas a >= b
 *   calibration  (Sec. "Calibration Pipeline": per-channel complex gains
 *                from a point-source model; least-squares reading)
 *       L = || V - G M G^H ||_F^2,  G = diag(g)
 *       grad_a = dL/dRe g_a + i dL/dIm g_a
 *              = -2 sum_b [ R_ab conj(M_ab) + conj(R_ba) M_ba ] g_b
 *   validity     (Sec. "CPU Data Collation": lost UDP packets and the
 *                weighting matrix; Sec. "Calibration Pipeline", weighting):
 *                spectrum s of antenna a is valid iff every input sample of
 *                its FIR window, s*P .. (s+T)*P - 1, arrived; the weight of
 *                a baseline is the number of spectra valid for both antennas
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* exp(-2 pi i m / P) from the exactly reduced integer angle m mod P */
static void twiddle(int64_t m, int64_t P, double *c, double *s)
{
    int64_t r = m % P;
    if (r < 0) r += P;
    double ang = -2.0 * ORC_PI * (double)r / (double)P;
    *c = cos(ang);
    *s = sin(ang);
}

/* ------------------------------------------------------------------------
 * Channeliser, polyphase form (Sec. "Polyphase Filterbank").
 *
 * x: int16 complex samples of one subband, element (n, i) at
 *    x[2*(n*row_stride + i) + {0: re, 1: im}], n < n_rows.
 * Computes spectra s in [s0, s1) of input `input`:
 *    y[2*((s - s0)*P + k) + {0,1}].
 * Valid mode: requires (s1 + T - 1) * P <= n_rows.  Returns 0 or -1.
 * ---------------------------------------------------------------------- */
int orc_ppf_stream(const int16_t *x, int64_t n_rows, int64_t row_stride, int64_t input,
                   const float *taps, int64_t P, int64_t T, int64_t s0, int64_t s1,
                   double *y)
{
    if (P <= 0 || T <= 0 || s0 < 0 || s1 < s0 || (s1 + T - 1) * P > n_rows) return -1;
    /* table of exp(-2 pi i (k p mod P) / P), each entry from twiddle() */
    double *wc = (double *)malloc(sizeof(double) * P * P);
    double *ws = (double *)malloc(sizeof(double) * P * P);
    if (!wc || !ws) { free(wc); free(ws); return -1; }
    for (int64_t k = 0; k < P; ++k)
        for (int64_t p = 0; p < P; ++p) twiddle(k * p, P, &wc[k * P + p], &ws[k * P + p]);
    int64_t s;
#pragma omp parallel for schedule(static)
    for (s = s0; s < s1; ++s) {
        double *ur = (double *)malloc(sizeof(double) * P);
        double *ui = (double *)malloc(sizeof(double) * P);
        /* FIR: one T-tap filter per branch p */
        for (int64_t p = 0; p < P; ++p) {
            double ar = 0.0, ai = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                double h = (double)taps[t * P + p];
                int64_t n = (s + t) * P + p;
                ar += h * (double)x[2 * (n * row_stride + input) + 0];
                ai += h * (double)x[2 * (n * row_stride + input) + 1];
            }
            ur[p] = ar;
            ui[p] = ai;
        }
        /* P-point DFT over the branches, summed directly */
        for (int64_t k = 0; k < P; ++k) {
            double yr = 0.0, yi = 0.0;
            for (int64_t p = 0; p < P; ++p) {
                const double c = wc[k * P + p], sn = ws[k * P + p];
                yr += ur[p] * c - ui[p] * sn;
                yi += ur[p] * sn + ui[p] * c;
            }
            y[2 * ((s - s0) * P + k) + 0] = yr;
            y[2 * ((s - s0) * P + k) + 1] = yi;
        }
        free(ur);
        free(ui);
    }
    free(wc);
    free(ws);
    return 0;
}

/* Same channeliser written as one windowed DFT of the M = P*T samples that
 * start at s*P:  y[s][k] = sum_{m<M} h[m] x[s*P+m] exp(-2 pi i k m / P).
 * It equals the polyphase form because exp(-2 pi i k (t*P+p)/P) does not
 * depend on t.  Used to cross-check the polyphase form. */
int orc_ppf_stream_direct(const int16_t *x, int64_t n_rows, int64_t row_stride, int64_t input,
                          const float *taps, int64_t P, int64_t T, int64_t s0, int64_t s1,
                          double *y)
{
    if (P <= 0 || T <= 0 || s0 < 0 || s1 < s0 || (s1 + T - 1) * P > n_rows) return -1;
    int64_t M = P * T;
    int64_t s;
#pragma omp parallel for schedule(static)
    for (s = s0; s < s1; ++s) {
        for (int64_t k = 0; k < P; ++k) {
            double yr = 0.0, yi = 0.0;
            for (int64_t m = 0; m < M; ++m) {
                int64_t n = s * P + m;
                double h = (double)taps[m];
                double xr = (double)x[2 * (n * row_stride + input) + 0];
                double xi = (double)x[2 * (n * row_stride + input) + 1];
                double c, sn;
                twiddle(k * m, P, &c, &sn);
                yr += h * (xr * c - xi * sn);
                yi += h * (xr * sn + xi * c);
            }
            y[2 * ((s - s0) * P + k) + 0] = yr;
            y[2 * ((s - s0) * P + k) + 1] = yi;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Requantiser to int8 (Sec. "LOFAR Digital Processing": the bit modes trade
 * word width for dynamic range).  Per real component:
 *    v = y * gain            (the exact product: two float32 values
 *                             multiply exactly in float64)
 *    q = clamp(rint(v), -127, 127)   (rint: nearest, ties to even)
 * so the product is rounded once, to the integer.  The symmetric range
 * keeps -q representable.
 * ---------------------------------------------------------------------- */
void orc_requant(const float *y, int64_t n, float gain, int8_t *q)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = (double)y[i] * (double)gain;
        double r = nearbyint(v);
        if (r > 127.0) r = 127.0;
        if (r < -127.0) r = -127.0;
        q[i] = (int8_t)r;
    }
}

/* ------------------------------------------------------------------------
 * Correlator (Sec. "Correlation Kernel"): time-integrated covariance of a
 * pair of receivers, V_ij = sum_s z_i(s) conj(z_j(s)).
 *
 * rows: complex samples [S][R][2] of R receivers; pairs: [n][2] receiver
 * indices (i, j); out: [n][2] (re, im).
 *   Re = sum (re_i re_j + im_i im_j),  Im = sum (im_i re_j - re_i im_j)
 * ---------------------------------------------------------------------- */
static void pair_f64(const double *rows, int64_t S, int64_t R, int64_t i, int64_t j,
                     double *out)
{
    double re = 0.0, im = 0.0;
    for (int64_t s = 0; s < S; ++s) {
        double ar = rows[2 * (s * R + i)], ai = rows[2 * (s * R + i) + 1];
        double br = rows[2 * (s * R + j)], bi = rows[2 * (s * R + j) + 1];
        re += ar * br + ai * bi;
        im += ai * br - ar * bi;
    }
    out[0] = re;
    out[1] = im;
}

void orc_xcorr_pairs_f64(const double *rows, int64_t S, int64_t R, int64_t n,
                         const int32_t *pairs, double *out)
{
    int64_t e;
#pragma omp parallel for schedule(static)
    for (e = 0; e < n; ++e) pair_f64(rows, S, R, pairs[2 * e], pairs[2 * e + 1], out + 2 * e);
}

/* Exact integer form for int8 samples, [S][R][2] int8 -> int64 sums. */
static void pair_i64(const int8_t *rows, int64_t S, int64_t R, int64_t i, int64_t j,
                     int64_t *out)
{
    int64_t re = 0, im = 0;
    for (int64_t s = 0; s < S; ++s) {
        int64_t ar = rows[2 * (s * R + i)], ai = rows[2 * (s * R + i) + 1];
        int64_t br = rows[2 * (s * R + j)], bi = rows[2 * (s * R + j) + 1];
        re += ar * br + ai * bi;
        im += ai * br - ar * bi;
    }
    out[0] = re;
    out[1] = im;
}

void orc_xcorr_pairs_i64(const int8_t *rows, int64_t S, int64_t R, int64_t n,
                         const int32_t *pairs, int64_t *out)
{
    int64_t e;
#pragma omp parallel for schedule(static)
    for (e = 0; e < n; ++e) pair_i64(rows, S, R, pairs[2 * e], pairs[2 * e + 1], out + 2 * e);
}

/* Whole lower triangle of one channel in the output layout
 * V[bl(a,b)][p][q][2], bl(a,b) = a(a+1)/2 + b for antennas a >= b, receivers
 * i = 2a+p, j = 2b+q.  flags: [Na] (1 = flagged) or NULL; a baseline that
 * touches a flagged antenna is 0 with weight 0, otherwise weight S.
 * z: [S][2*Na][2]. */
void orc_xcorr_f64(const double *z, int64_t S, int64_t Na, const uint8_t *flags,
                   double *V, int32_t *W)
{
    int64_t R = 2 * Na;
    int64_t a;
#pragma omp parallel for schedule(dynamic, 1)
    for (a = 0; a < Na; ++a) {
        for (int64_t b = 0; b <= a; ++b) {
            int64_t bl = a * (a + 1) / 2 + b;
            int flagged = flags && (flags[a] || flags[b]);
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) {
                    double re = 0.0, im = 0.0;
                    if (!flagged) {
                        double o[2];
                        pair_f64(z, S, R, 2 * a + p, 2 * b + q, o);
                        re = o[0];
                        im = o[1];
                    }
                    V[2 * ((bl * 2 + p) * 2 + q) + 0] = re;
                    V[2 * ((bl * 2 + p) * 2 + q) + 1] = im;
                }
            if (W) W[bl] = flagged ? 0 : (int32_t)S;
        }
    }
}

/* Integer whole-triangle form; returns -1 if any |sum| reaches 2^31 (the
 * int32 accumulator of the device path would not hold it), else 0. */
int orc_xcorr_i64(const int8_t *z, int64_t S, int64_t Na, const uint8_t *flags,
                  int64_t *V, int32_t *W)
{
    int64_t R = 2 * Na;
    int bad = 0;
    int64_t a;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (a = 0; a < Na; ++a) {
        for (int64_t b = 0; b <= a; ++b) {
            int64_t bl = a * (a + 1) / 2 + b;
            int flagged = flags && (flags[a] || flags[b]);
            for (int p = 0; p < 2; ++p)
                for (int q = 0; q < 2; ++q) {
                    int64_t o[2] = {0, 0};
                    if (!flagged) pair_i64(z, S, R, 2 * a + p, 2 * b + q, o);
                    if (o[0] >= 2147483648LL || o[0] <= -2147483648LL ||
                        o[1] >= 2147483648LL || o[1] <= -2147483648LL) bad = 1;
                    V[2 * ((bl * 2 + p) * 2 + q) + 0] = o[0];
                    V[2 * ((bl * 2 + p) * 2 + q) + 1] = o[1];
                }
            if (W) W[bl] = flagged ? 0 : (int32_t)S;
        }
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * Gain-calibration loss and gradient (Sec. "Calibration Pipeline": per
 * channel amplitude and phase gains from a point-source sky model, XX and
 * YY).  Least-squares reading: L = sum_{a,b} |R_ab|^2 over the full
 * Hermitian matrix, R = V - G M G^H.
 *
 * V, M: float32 [P][Nbl][2][2][2] lower triangles (the correlator layout;
 *       XX = [0][0], YY = [1][1]); the upper triangle is the conjugate.
 * g:    float32 [P][Na][2][2] complex gain per channel, antenna, pol.
 * loss: [P][2];  grad: [P][Na][2][2] = dL/dRe g + i dL/dIm g, or NULL.
 *
 * Weighted form (Sec. "Real-time Flagging, Calibration and Imaging": the
 * calibration works on the flagged visibilities, re-weighted for lost
 * data): with real weights w_ab = w_ba >= 0 per stored baseline and
 * polarisation, double [P][Nbl][2] (NULL = all 1),
 *   L = sum_{a,b} w_ab |R_ab|^2,
 *   grad_a = -2 sum_b [w_ab R_ab conj(M_ab) + w_ba conj(R_ba) M_ba] g_b.
 * A flagged baseline has weight 0.
 * ---------------------------------------------------------------------- */
int orc_cal_loss_grad_w(const float *V, const float *M, const double *w, const float *g, int64_t Na,
                        int64_t P, double *loss, double *grad)
{
    int64_t nbl = Na * (Na + 1) / 2;
    int64_t job;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (job = 0; job < 2 * P; ++job) {
        int64_t ch = job / 2, pol = job % 2;
        double *Vr = (double *)malloc(sizeof(double) * 2 * Na * Na);
        double *Mr = (double *)malloc(sizeof(double) * 2 * Na * Na);
        double *Rr = (double *)malloc(sizeof(double) * 2 * Na * Na);
        double *Wr = (double *)malloc(sizeof(double) * Na * Na);
        if (!Vr || !Mr || !Rr || !Wr) { err = 1; free(Vr); free(Mr); free(Rr); free(Wr); continue; }
        /* Hermitian completion of the stored lower triangle (the weights
         * are symmetric) */
        for (int64_t a = 0; a < Na; ++a)
            for (int64_t b = 0; b <= a; ++b) {
                int64_t off = 2 * (((ch * nbl + a * (a + 1) / 2 + b) * 2 + pol) * 2 + pol);
                double vr = V[off], vi = V[off + 1], mr = M[off], mi = M[off + 1];
                Vr[2 * (a * Na + b)] = vr;  Vr[2 * (a * Na + b) + 1] = vi;
                Vr[2 * (b * Na + a)] = vr;  Vr[2 * (b * Na + a) + 1] = -vi;
                Mr[2 * (a * Na + b)] = mr;  Mr[2 * (a * Na + b) + 1] = mi;
                Mr[2 * (b * Na + a)] = mr;  Mr[2 * (b * Na + a) + 1] = -mi;
                if (a == b) { Vr[2 * (a * Na + a) + 1] = vi; Mr[2 * (a * Na + a) + 1] = mi; }
                Wr[a * Na + b] = Wr[b * Na + a] = w ? w[(ch * nbl + a * (a + 1) / 2 + b) * 2 + pol] : 1.0;
            }
        /* R_ab = V_ab - g_a M_ab conj(g_b);  L = sum |R_ab|^2 */
        double L = 0.0;
        for (int64_t a = 0; a < Na; ++a) {
            double gar = g[2 * ((ch * Na + a) * 2 + pol)], gai = g[2 * ((ch * Na + a) * 2 + pol) + 1];
            for (int64_t b = 0; b < Na; ++b) {
                double gbr = g[2 * ((ch * Na + b) * 2 + pol)], gbi = g[2 * ((ch * Na + b) * 2 + pol) + 1];
                double mr = Mr[2 * (a * Na + b)], mi = Mr[2 * (a * Na + b) + 1];
                /* t = g_a * M_ab */
                double tr = gar * mr - gai * mi, ti = gar * mi + gai * mr;
                /* w = t * conj(g_b) */
                double wr = tr * gbr + ti * gbi, wi = ti * gbr - tr * gbi;
                double rr = Vr[2 * (a * Na + b)] - wr, ri = Vr[2 * (a * Na + b) + 1] - wi;
                Rr[2 * (a * Na + b)] = rr;
                Rr[2 * (a * Na + b) + 1] = ri;
                L += Wr[a * Na + b] * (rr * rr + ri * ri);
            }
        }
        loss[ch * 2 + pol] = L;
        if (grad) {
            for (int64_t a = 0; a < Na; ++a) {
                double sr = 0.0, si = 0.0;
                for (int64_t b = 0; b < Na; ++b) {
                    /* c = R_ab conj(M_ab) + conj(R_ba) M_ba */
                    double rr = Rr[2 * (a * Na + b)], ri = Rr[2 * (a * Na + b) + 1];
                    double mr = Mr[2 * (a * Na + b)], mi = Mr[2 * (a * Na + b) + 1];
                    double wab = Wr[a * Na + b], wba = Wr[b * Na + a];
                    double cr = wab * (rr * mr + ri * mi), ci = wab * (ri * mr - rr * mi);
                    double r2r = Rr[2 * (b * Na + a)], r2i = -Rr[2 * (b * Na + a) + 1];
                    double m2r = Mr[2 * (b * Na + a)], m2i = Mr[2 * (b * Na + a) + 1];
                    cr += wba * (r2r * m2r - r2i * m2i);
                    ci += wba * (r2r * m2i + r2i * m2r);
                    double gbr = g[2 * ((ch * Na + b) * 2 + pol)], gbi = g[2 * ((ch * Na + b) * 2 + pol) + 1];
                    sr += cr * gbr - ci * gbi;
                    si += cr * gbi + ci * gbr;
                }
                grad[2 * ((ch * Na + a) * 2 + pol)] = -2.0 * sr;
                grad[2 * ((ch * Na + a) * 2 + pol) + 1] = -2.0 * si;
            }
        }
        free(Vr); free(Mr); free(Rr); free(Wr);
    }
    return err ? -1 : 0;
}

int orc_cal_loss_grad(const float *V, const float *M, const float *g, int64_t Na, int64_t P,
                      double *loss, double *grad)
{
    return orc_cal_loss_grad_w(V, M, NULL, g, Na, P, loss, grad);
}

/* ------------------------------------------------------------------------
 * Fine channeliser with delay and bandpass compensation and channel
 * integration (Sec. "Polyphase Filterbank": a 256-channel bank; Sec.
 * "Delay, Bandpass Compensation and Transpose Kernel": cable delays applied
 * as phase rotations of the channelised data, a fixed real weight per
 * channel against the first-stage bandpass, then channels integrated to the
 * desired resolution).  Readings:
 *   fine spectra  y[s][k] by the polyphase definition above with P = Pf;
 *   channel k (natural order) sits at sky frequency
 *       nu_k = nu_c + f_k,  f_k = (k < Pf/2 ? k : k - Pf) * df;
 *   a signal that reaches input i tau_i late carries exp(-2 pi i nu tau_i)
 *   in complex baseband, so the compensation multiplies by
 *       exp(+2 pi i nu_k tau_i);
 *   bandpass: times the real weight w[k];
 *   integration: the coherent sum of the R adjacent fine channels
 *       zc[s][c] = sum_{j<R} w[R c + j] exp(2 pi i nu_{Rc+j} tau_i) y[s][R c + j],
 *   c < Pf / R in natural order (so coarse channel c covers the signed fine
 *   offsets R c' + {0 .. R-1}, c' the signed index of c).
 * Output zc[2*((s - s0)*(Pf/R) + c) + {0,1}].  Returns 0 or -1.
 * ---------------------------------------------------------------------- */
int orc_fine_channelise(const int16_t *x, int64_t n_rows, int64_t row_stride, int64_t input,
                        const float *taps, int64_t Pf, int64_t T, int64_t s0, int64_t s1,
                        double tau, double nu_c, double df, const float *w, int64_t R, double *zc)
{
    if (R <= 0 || Pf % R != 0) return -1;
    const int64_t Pc = Pf / R, n = s1 - s0;
    double *y = (double *)malloc(sizeof(double) * 2 * (n > 0 ? n : 1) * Pf);
    if (!y) return -1;
    if (orc_ppf_stream(x, n_rows, row_stride, input, taps, Pf, T, s0, s1, y) != 0) {
        free(y);
        return -1;
    }
    /* compensation factor of each fine channel */
    double *fr = (double *)malloc(sizeof(double) * Pf);
    double *fi = (double *)malloc(sizeof(double) * Pf);
    if (!fr || !fi) { free(y); free(fr); free(fi); return -1; }
    for (int64_t k = 0; k < Pf; ++k) {
        const double fk = (double)(k < Pf / 2 ? k : k - Pf) * df;
        const double ang = 2.0 * ORC_PI * (nu_c + fk) * tau;
        fr[k] = (double)w[k] * cos(ang);
        fi[k] = (double)w[k] * sin(ang);
    }
    for (int64_t s = 0; s < n; ++s)
        for (int64_t c = 0; c < Pc; ++c) {
            double ar = 0.0, ai = 0.0;
            for (int64_t j = 0; j < R; ++j) {
                const int64_t k = R * c + j;
                const double yr = y[2 * (s * Pf + k)], yi = y[2 * (s * Pf + k) + 1];
                ar += fr[k] * yr - fi[k] * yi;
                ai += fr[k] * yi + fi[k] * yr;
            }
            zc[2 * (s * Pc + c)] = ar;
            zc[2 * (s * Pc + c) + 1] = ai;
        }
    free(y); free(fr); free(fi);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Validity of channelised spectra after lost packets (Sec. "CPU Data
 * Collation": the correlator handles lost UDP packets and produces a
 * weighting matrix with the visibilities).
 *
 * pkt[k * Na + a] != 0 when packet k of antenna a arrived; a packet carries
 * Q consecutive input samples (sample n is in packet n / Q; samples past the
 * last packet count as lost).  Spectrum s of a bank with P samples per
 * spectrum and T taps reads samples s*P .. (s+T)*P - 1 and is valid iff all
 * of them arrived.  Antennas a0 .. a1-1; v[(a - a0) * S + s] = 0 or 1.
 * ------------------------------------------------------------------------- */
void orc_spectrum_validity(const uint8_t *pkt, int64_t n_pk, int64_t Na, int64_t Q, int64_t P,
                           int64_t T, int64_t S, int64_t a0, int64_t a1, uint8_t *v)
{
    int64_t a;
#pragma omp parallel for schedule(static)
    for (a = a0; a < a1; ++a)
        for (int64_t s = 0; s < S; ++s) {
            int ok = 1;
            for (int64_t n = s * P; n < (s + T) * P && ok; ++n) {
                const int64_t k = n / Q;
                if (k >= n_pk || !pkt[k * Na + a]) ok = 0;
            }
            v[(a - a0) * S + s] = (uint8_t)ok;
        }
}

/* Weighting matrix of one subband: W[bl(a,b)] = number of spectra s < S
 * valid for both antennas (v[a * S_stride + s]), 0 when either antenna is
 * flagged (flags may be NULL). */
void orc_validity_weights(const uint8_t *v, int64_t Na, int64_t S_stride, int64_t S,
                          const uint8_t *flags, int32_t *W)
{
    int64_t a;
#pragma omp parallel for schedule(dynamic, 4)
    for (a = 0; a < Na; ++a)
        for (int64_t b = 0; b <= a; ++b) {
            int64_t n = 0;
            if (!(flags && (flags[a] || flags[b])))
                for (int64_t s = 0; s < S; ++s) n += v[a * S_stride + s] && v[b * S_stride + s];
            W[a * (a + 1) / 2 + b] = (int32_t)n;
        }
}
