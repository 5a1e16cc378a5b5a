/*
 * Host-only driver that runs every function of the CPU oracle on small and
 * degenerate inputs, built with the address and undefined-behaviour
 * sanitizers (test infrastructure; see test_oracle_sanitizers.py).  Besides
 * running clean under the sanitizers it checks a few identities, so that a
 * run that silently computes nothing does not pass:
 *   - the polyphase and windowed-DFT forms of the channeliser agree;
 *   - the pair and whole-triangle correlators agree, in float and integer;
 *   - an impossible range returns -1;
 *   - the calibration gradient is zero at noise-free gains.
 * Exit status 0 on success; a message and 1 otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_ppf_stream(const int16_t *, int64_t, int64_t, int64_t, const float *, int64_t, int64_t, int64_t,
                   int64_t, double *);
int orc_ppf_stream_direct(const int16_t *, int64_t, int64_t, int64_t, const float *, int64_t, int64_t, int64_t,
                          int64_t, double *);
void orc_requant(const float *, int64_t, float, int8_t *);
void orc_xcorr_pairs_f64(const double *, int64_t, int64_t, int64_t, const int32_t *, double *);
void orc_xcorr_pairs_i64(const int8_t *, int64_t, int64_t, int64_t, const int32_t *, int64_t *);
void orc_xcorr_f64(const double *, int64_t, int64_t, const uint8_t *, double *, int32_t *);
int orc_xcorr_i64(const int8_t *, int64_t, int64_t, const uint8_t *, int64_t *, int32_t *);
int orc_cal_loss_grad(const float *, const float *, const float *, int64_t, int64_t, double *, double *);
int orc_cal_loss_grad_w(const float *, const float *, const double *, const float *, int64_t, int64_t, double *,
                        double *);
int orc_fine_channelise(const int16_t *, int64_t, int64_t, int64_t, const float *, int64_t, int64_t, int64_t,
                        int64_t, double, double, double, const float *, int64_t, double *);
void orc_spectrum_validity(const uint8_t *, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                           int64_t, uint8_t *);
void orc_validity_weights(const uint8_t *, int64_t, int64_t, int64_t, const uint8_t *, int32_t *);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void)
{
    /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545F4914F6CDD1Dull) >> 32);
}
static double uniform(void) { return (next_u32() + 0.5) / 4294967296.0; }

#define CHECK(c, msg)                                        \
    do {                                                     \
        if (!(c)) {                                          \
            fprintf(stderr, "check failed: %s\n", msg);      \
            return 1;                                        \
        }                                                    \
    } while (0)

static int channeliser(void)
{
    const int64_t P = 8, T = 4, S = 5, R = 3, L = (S + T - 1) * P;
    int16_t *x = malloc(sizeof(int16_t) * 2 * L * R);
    float *h = malloc(sizeof(float) * P * T);
    double *a = malloc(sizeof(double) * 2 * S * P), *b = malloc(sizeof(double) * 2 * S * P);
    for (int64_t n = 0; n < 2 * L * R; ++n) x[n] = (int16_t)((int)(next_u32() % 20001) - 10000);
    for (int64_t m = 0; m < P * T; ++m) h[m] = (float)(uniform() - 0.5);
    for (int64_t i = 0; i < R; ++i) {
        CHECK(orc_ppf_stream(x, L, R, i, h, P, T, 0, S, a) == 0, "ppf range");
        CHECK(orc_ppf_stream_direct(x, L, R, i, h, P, T, 0, S, b) == 0, "direct range");
        for (int64_t n = 0; n < 2 * S * P; ++n) CHECK(fabs(a[n] - b[n]) <= 1e-9 * (1 + fabs(b[n])), "forms agree");
    }
    CHECK(orc_ppf_stream(x, L, R, 0, h, P, T, 0, S + 1, a) == -1, "range past the input is refused");
    CHECK(orc_ppf_stream(x, L, R, 0, h, P, T, 2, 2, a) == 0, "empty range");
    /* fine channeliser: P = 8 branches integrated 2:1 */
    double *z = malloc(sizeof(double) * 2 * S * (P / 2));
    float w[8];
    for (int k = 0; k < 8; ++k) w[k] = (float)(0.5 + uniform());
    CHECK(orc_fine_channelise(x, L, R, 1, h, P, T, 0, S, 3e-9, 60e6, 195312.5 / P, w, 2, z) == 0, "fine");
    CHECK(orc_fine_channelise(x, L, R, 1, h, P, T, 0, S, 3e-9, 60e6, 195312.5 / P, w, 3, z) == -1,
          "fine ratio must divide the channels");
    CHECK(orc_fine_channelise(x, L, R, 1, h, P, T, 0, 0, 0.0, 60e6, 1.0, w, 2, z) == 0, "fine empty");
    float y[6] = {2.5f, -2.5f, 300.0f, -300.0f, 0.49f, 1e30f};
    int8_t q[6];
    orc_requant(y, 6, 1.0f, q);
    CHECK(q[0] == 2 && q[1] == -2 && q[2] == 127 && q[3] == -127 && q[4] == 0 && q[5] == 127, "requant");
    orc_requant(y, 0, 1.0f, q);
    free(x); free(h); free(a); free(b); free(z);
    return 0;
}

static int correlator(void)
{
    const int64_t S = 9, Na = 3, R = 2 * Na, nbl = Na * (Na + 1) / 2;
    double *zf = malloc(sizeof(double) * 2 * S * R);
    int8_t *zi = malloc(2 * S * R);
    for (int64_t n = 0; n < 2 * S * R; ++n) {
        zi[n] = (int8_t)((int)(next_u32() % 255) - 127);
        zf[n] = zi[n];
    }
    double *Vf = malloc(sizeof(double) * nbl * 8);
    int64_t *Vi = malloc(sizeof(int64_t) * nbl * 8);
    int32_t W[6], W2[6];
    uint8_t flags[3] = {0, 1, 0};
    orc_xcorr_f64(zf, S, Na, NULL, Vf, W);
    CHECK(orc_xcorr_i64(zi, S, Na, flags, Vi, W2) == 0, "int range");
    int32_t pairs[2 * 36];
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) { pairs[2 * (i * R + j)] = i; pairs[2 * (i * R + j) + 1] = j; }
    double of[2 * 36];
    int64_t oi[2 * 36];
    orc_xcorr_pairs_f64(zf, S, R, 36, pairs, of);
    orc_xcorr_pairs_i64(zi, S, R, 36, pairs, oi);
    for (int64_t a = 0; a < Na; ++a)
        for (int64_t b = 0; b <= a; ++b)
            for (int p = 0; p < 2; ++p)
                for (int qq = 0; qq < 2; ++qq) {
                    const int64_t bl = a * (a + 1) / 2 + b, e = (2 * a + p) * R + 2 * b + qq;
                    const int64_t o = 2 * ((bl * 2 + p) * 2 + qq);
                    CHECK(Vf[o] == of[2 * e] && Vf[o + 1] == of[2 * e + 1], "float pair = triangle");
                    const int hit = flags[a] || flags[b];
                    CHECK(Vi[o] == (hit ? 0 : oi[2 * e]) && Vi[o + 1] == (hit ? 0 : oi[2 * e + 1]),
                          "int pair = triangle, flags zero");
                    CHECK(W2[bl] == (hit ? 0 : S) && W[bl] == S, "weights");
                }
    orc_xcorr_f64(zf, 0, Na, NULL, Vf, W);             /* no spectra: all zero */
    for (int64_t n = 0; n < nbl * 8; ++n) CHECK(Vf[n] == 0.0, "empty integration");
    free(zf); free(zi); free(Vf); free(Vi);
    return 0;
}

static int calibration(void)
{
    const int64_t Na = 4, P = 2, nbl = Na * (Na + 1) / 2;
    float *V = calloc(P * nbl * 8, sizeof(float)), *M = calloc(P * nbl * 8, sizeof(float));
    float *g = malloc(sizeof(float) * P * Na * 4);
    double loss[4], *grad = malloc(sizeof(double) * P * Na * 4);
    /* gains on a grid of powers of two: g_a M_ab conj(g_b) is exact in float */
    for (int64_t n = 0; n < P * Na * 4; ++n) g[n] = (float)((int)(next_u32() % 5) - 2) * 0.5f;
    for (int64_t n = 0; n < P * Na * 2; ++n)
        if (g[2 * n] == 0 && g[2 * n + 1] == 0) g[2 * n] = 1.0f;
    for (int64_t ch = 0; ch < P; ++ch)
        for (int64_t a = 0; a < Na; ++a)
            for (int64_t b = 0; b <= a; ++b)
                for (int pol = 0; pol < 2; ++pol) {
                    const int64_t o = 2 * (((ch * nbl + a * (a + 1) / 2 + b) * 2 + pol) * 2 + pol);
                    const float mr = (float)((int)(next_u32() % 9) - 4), mi = a == b ? 0.0f : (float)((int)(next_u32() % 9) - 4);
                    M[o] = mr;
                    M[o + 1] = mi;
                    const float *ga = g + 2 * ((ch * Na + a) * 2 + pol), *gb = g + 2 * ((ch * Na + b) * 2 + pol);
                    const float tr = ga[0] * mr - ga[1] * mi, ti = ga[0] * mi + ga[1] * mr;
                    V[o] = tr * gb[0] + ti * gb[1];
                    V[o + 1] = ti * gb[0] - tr * gb[1];
                }
    CHECK(orc_cal_loss_grad(V, M, g, Na, P, loss, grad) == 0, "cal");
    for (int k = 0; k < 4; ++k) CHECK(loss[k] == 0.0, "noise-free loss is zero");
    for (int64_t n = 0; n < P * Na * 4; ++n) CHECK(grad[n] == 0.0, "noise-free gradient is zero");
    CHECK(orc_cal_loss_grad(V, M, g, Na, P, loss, NULL) == 0, "loss only");
    {   /* weighted form: noise-free data stay at zero loss and gradient */
        const int64_t nbl = Na * (Na + 1) / 2;
        double *w = malloc(sizeof(double) * P * nbl * 2);
        for (int64_t n = 0; n < P * nbl * 2; ++n) w[n] = (double)(n % 3);
        CHECK(orc_cal_loss_grad_w(V, M, w, g, Na, P, loss, grad) == 0, "weighted cal");
        for (int k = 0; k < 4; ++k) CHECK(loss[k] == 0.0, "weighted noise-free loss is zero");
        for (int64_t n = 0; n < P * Na * 4; ++n) CHECK(grad[n] == 0.0, "weighted noise-free gradient is zero");
        free(w);
    }
    free(V); free(M); free(g); free(grad);
    return 0;
}

static int validity(void)
{
    const int64_t Na = 3, Q = 4, P = 8, T = 2, S = 6, n_pk = (S + T - 1) * P / Q;
    uint8_t *pkt = malloc(n_pk * Na), v[3 * 6];
    for (int64_t n = 0; n < n_pk * Na; ++n) pkt[n] = 1;
    pkt[5 * Na + 1] = 0;                               /* packet 5 of antenna 1: samples 20..23 */
    orc_spectrum_validity(pkt, n_pk, Na, Q, P, T, S, 0, Na, v);
    for (int64_t s = 0; s < S; ++s) {
        /* spectrum s reads samples 8s .. 8s + 15 */
        const int lost = 8 * s <= 23 && 20 <= 8 * s + 15;
        CHECK(v[0 * S + s] == 1 && v[2 * S + s] == 1 && v[1 * S + s] == !lost, "validity");
    }
    orc_spectrum_validity(pkt, n_pk - 1, Na, Q, P, T, S, 1, 2, v);   /* short stream: tail lost */
    CHECK(v[S - 1] == 0, "samples past the last packet are lost");
    int32_t W[6];
    uint8_t flags[3] = {0, 0, 1};
    orc_spectrum_validity(pkt, n_pk, Na, Q, P, T, S, 0, Na, v);
    orc_validity_weights(v, Na, S, S, flags, W);
    CHECK(W[0] == S && W[1] == S - 2 && W[2] == S - 2 && W[3] == 0 && W[4] == 0 && W[5] == 0, "weights");
    free(pkt);
    return 0;
}

int main(void)
{
    if (channeliser() || correlator() || calibration() || validity()) return 1;
    printf("oracle sanitizer driver ok\n");
    return 0;
}
