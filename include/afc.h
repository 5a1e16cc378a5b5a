/*
 * afc.h -- C ABI of an MI355X (gfx950) FX correlator for AARTFAAC-style
 * all-sky monitors (arXiv 1609.04205).
 *
 * The library implements the correlator's data-parallel hot path:
 *   afc_channelise      polyphase filter bank (FIR + FFT) with the corner turn
 *                       to the correlator's input-major layout, optional
 *                       requantisation to int8 or conversion to fp16
 *   afc_correlate       X-engine: lower triangle of the time-integrated
 *                       Hermitian visibility matrix per channel, on MFMA
 *   afc_calibrate_grad  gain-calibration loss ||V - G M G^H||_F^2 and its
 *                       gradient with respect to the complex gains
 *   afc_plan_*          batching form: many subbands with their own
 *                       integration length, sample type and antenna flags in
 *                       one graph of one channeliser launch and one
 *                       correlator launch per sample-type family, tile shape
 *                       from a measured tuner
 *
 * Conventions (all entry points):
 *   - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *     owns every buffer; the library never allocates or frees device memory
 *     on these calls, except the plans: afc_plan_create allocates the plan's
 *     tables, and an afc_plan_launch that captures a new graph allocates that
 *     graph's small item table (see afc_plan_launch).
 *   - Every call is asynchronous on `stream` (a hipStream_t; 0 = null stream).
 *     Argument errors are found on the host before anything is launched and
 *     return a negative afc_status; afc_last_error() then holds a message
 *     (thread-local).  Faults inside kernels surface at the caller's next
 *     synchronisation of the stream.  No C++ exception crosses the ABI.
 *   - Receivers: an antenna has n_pols = 2 polarisations; receiver (input)
 *     i = 2*a + p (p = 0 "X", 1 "Y"), N = 2*n_antennas receivers.
 *   - Baselines: antennas a >= b, bl(a, b) = a*(a+1)/2 + b,
 *     Nbl = n_antennas*(n_antennas+1)/2.
 *
 * Two amendments to the interface first proposed for this library:
 *   - The channelised array z is [B][P][ceil(S/8)][N][8] (blocks of 8
 *     spectra per receiver) instead of [B][P][S][Na][Np].  Both the
 *     channeliser's stores and the correlator's operand loads then move whole
 *     64-byte (int8: 16-byte) runs per receiver; spectra >= S in the last
 *     block are zero.  Receiver i = 2a + p is the same index in both forms.
 *   - afc_calibrate_grad takes a caller-provided workspace (per-tile partial
 *     sums), so that the gradient is reduced in a fixed order without
 *     atomics and the call allocates nothing.
 */
#ifndef AFC_H
#define AFC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AFC_API __attribute__((visibility("default")))

typedef enum {
    AFC_OK = 0,
    AFC_ERR_INVALID = -1,      /* a NULL pointer, a bad size or layout        */
    AFC_ERR_UNSUPPORTED = -2,  /* valid in principle, not built (e.g. P != 64) */
    AFC_ERR_HIP = -3,          /* a HIP runtime call failed                    */
    AFC_ERR_WORKSPACE = -4     /* workspace missing or too small               */
} afc_status;

typedef enum {
    AFC_F32 = 0,               /* complex float32  (8 bytes per sample)        */
    AFC_F16 = 1,               /* complex float16  (4 bytes per sample)        */
    AFC_I8 = 2                 /* complex int8 in [-127, 127] (2 bytes)        */
} afc_dtype;

/* Spectra per block in the channelised layout (see afc_channelise). */
#define AFC_SPECTRUM_BLOCK 8
/* Largest subband count one call accepts. */
#define AFC_MAX_SUBBANDS 256

/* Problem shape, following the paper's statement of the correlator's input:
 * subbanded complex voltages of each polarisation of every antenna
 * (Sec. "The AARTFAAC Correlator"), channelised by a T-tap, P-channel
 * polyphase filter bank (Sec. "Polyphase Filterbank") and integrated over
 * n_spectra spectra (about 1 s at P = 64: 3051 spectra). */
typedef struct afc_dims {
    int32_t n_antennas;   /* Na >= 1                                          */
    int32_t n_pols;       /* must be 2                                         */
    int32_t n_subbands;   /* B, 1 .. AFC_MAX_SUBBANDS                          */
    int32_t n_channels;   /* P, must be 64                                     */
    int32_t n_taps;       /* T, must be 16                                     */
    int32_t n_spectra;    /* S >= 1 (the maximum over subbands when batched)   */
} afc_dims;

/* Bytes of the channelised array z for `d` and sample type `dt`:
 * B * P * ceil(S/8) * N * 8 * sample_bytes.  0 if `d` is invalid. */
AFC_API size_t afc_channelised_bytes(const afc_dims* d, afc_dtype dt);

/* Bytes of the visibility array for `d`: B * P * Nbl * 4 * 8 (both float2
 * and int2 samples are 8 bytes). */
AFC_API size_t afc_visibility_bytes(const afc_dims* d);

/* ---------------------------------------------------------------------------
 * afc_channelise -- polyphase filter bank per receiver and subband
 * (Sec. "Polyphase Filterbank": a bank of 16-tap FIR filters followed by a
 * complex FFT, here P = 64 channels; Sec. "Delay, Bandpass Compensation and
 * Transpose Kernel": the corner turn from channel-major to receiver-major is
 * fused into the store).
 *
 *   u[s][p] = sum_{t<T} taps[t*P + p] * x[(s+t)*P + p]          (FIR, p < P)
 *   y[s][k] = sum_{p<P} u[s][p] * exp(-2 pi i k p / P)          (FFT, k < P)
 *
 * Channel k is the natural FFT order (k = 0 is the subband centre, k >= P/2
 * are negative frequency offsets); no normalisation.
 *
 * x     int16 [B][L][N][2], L = (S + T - 1) * P rows of N receivers, re/im
 *       interleaved (time-major; all receivers of a time sample contiguous).
 *       Rows beyond L are not read.
 * taps  float [T*P], in the order taps[t*P + p].  Any real finite filter; the
 *       FIR uses each tap to 22 significant bits (after a power-of-two scale)
 *       with exact products summed in float32, the FFT float32.
 * out   [B][P][Sb][N][8] complex of out_dtype, Sb = ceil(S/8): spectrum s of
 *       receiver i in channel k of subband b sits at block s/8, slot s%8.
 *       Slots of spectra >= S are written as zero.  Size from
 *       afc_channelised_bytes().
 * out_dtype AFC_F32: the float32 value.  AFC_F16: rounded to nearest even.
 *       AFC_I8: per real component q = clamp(rint(y * requant_gain), -127,
 *       127), the exact product rounded once, ties to even
 *       (Sec. "LOFAR Digital Processing": fewer bits per sample for more
 *       subbands); requant_gain is ignored for the other types.
 * Limits: P = 64, T = 16, n_pols = 2, L*N*2 < 2^31 per subband.
 * ------------------------------------------------------------------------- */
AFC_API int afc_channelise(const afc_dims* d, const int16_t* x, const float* taps,
                           afc_dtype out_dtype, float requant_gain, void* out,
                           hipStream_t stream);

/* ---------------------------------------------------------------------------
 * afc_channelise_fine -- the paper's channeliser configuration: a 256-channel
 * polyphase filter bank (Sec. "Polyphase Filterbank": 256 16-tap FIR filters
 * and a 256-point complex FFT), fixed cable-delay compensation as phase
 * rotations and a fixed real weight per channel against the first-stage
 * bandpass ripple, then integration of adjacent channels to the output
 * resolution and the corner turn (Sec. "Delay, Bandpass Compensation and
 * Transpose Kernel").  Per receiver i of subband b:
 *
 *   u[s][p] = sum_{t<16} taps[t*256 + p] * x[(s+t)*256 + p]     (p < 256)
 *   y[s][k] = sum_{p<256} u[s][p] * exp(-2 pi i k p / 256)      (k < 256)
 *   f_k     = (k < 128 ? k : k - 256) * subband_width_hz / 256
 *   z[s][c] = sum_{j<4} bandpass[4c+j] * exp(2 pi i (center_hz[b] + f_{4c+j})
 *                                              * delays[i]) * y[s][4c+j]
 *
 * for c < 64: output channel c is the coherent sum of fine channels
 * 4c .. 4c+3 in natural FFT order.  A spectrum s spans 256 input samples, so
 * z holds d->n_spectra spectra of 64 channels and is laid out, typed and
 * sized exactly as afc_channelise's output (afc_correlate takes it as is).
 *
 * d        n_channels = 64 (the output channels), n_taps = 16, n_spectra = S
 *          (256-sample spectra).
 * x        int16 [B][L][N][2], L = (S + 15) * 256 rows, as in afc_channelise.
 * taps     float [16*256] in the order taps[t*256 + p].
 * delays   double [N] (device), seconds, per receiver; positive = the signal
 *          arrives late.
 * bandpass float [256] (device), real weight per fine channel k (natural order).
 * center_hz  double [B] (host), sky frequency of each subband's centre.
 * subband_width_hz  > 0 (195312.5 for the 200 MHz sample clock).
 * out_dtype, requant_gain  as in afc_channelise.
 * workspace  device buffer of afc_channelise_fine_workspace_bytes(d) bytes:
 *          the tables of exp(-2 pi i m / 256), of bandpass-weighted delay
 *          phases per (receiver, fine channel) and of centre-frequency phases
 *          per (subband, receiver), recomputed in float64 on every call.
 *          Calls sharing one workspace on different streams race.
 * out      as afc_channelise, afc_channelised_bytes(d, out_dtype) bytes.
 * Limits: L*N*2 < 2^31 per subband; other limits as afc_channelise.
 * ------------------------------------------------------------------------- */
AFC_API size_t afc_channelise_fine_workspace_bytes(const afc_dims* d);
AFC_API int afc_channelise_fine(const afc_dims* d, const int16_t* x, const float* taps,
                                const double* delays, const float* bandpass,
                                const double* center_hz, double subband_width_hz,
                                afc_dtype out_dtype, float requant_gain, void* workspace,
                                void* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * afc_correlate -- X-engine (Sec. "Correlation Kernel": only one triangle of
 * the Hermitian covariance matrix is computed, per channel, and the
 * visibilities are accumulated over the integration; Sec. "CPU Data
 * Collation": a weighting matrix accompanies the visibilities).
 *
 *   V[b][k][bl(a,c)][p][q] = sum_{s < S_b} z_i(s) * conj(z_j(s)),
 *                            i = 2a+p, j = 2c+q, a >= c
 *
 * z        channelised samples in the afc_channelise layout, type in_dtype;
 *          int8 samples must lie in [-127, 127].
 * n_spectra_per_sb  host int32 [B] with 1 <= S_b <= d->n_spectra, or NULL
 *          (all S).  Spectra >= S_b of subband b are ignored whatever they
 *          hold.
 * flags    uint8 [B][Na] (nonzero = flagged antenna) or NULL.  A baseline
 *          that touches a flagged antenna gets V = 0 and weight 0.
 * vis      [B][P][Nbl][2][2] complex: float2 for AFC_F32 / AFC_F16 (float32
 *          accumulation), int2 for AFC_I8 (exact int32 accumulation; exact
 *          while 2 * 127^2 * S_b < 2^31), 16-byte aligned (else
 *          AFC_ERR_INVALID).  Autocorrelations (i == j) have imaginary part
 *          exactly 0.
 * weights  int32 [B][Nbl] or NULL: S_b, or 0 for flagged baselines.
 * ------------------------------------------------------------------------- */
AFC_API int afc_correlate(const afc_dims* d, afc_dtype in_dtype, const void* z,
                          const int32_t* n_spectra_per_sb, const uint8_t* flags,
                          void* vis, int32_t* weights, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Lost packets and the weighting matrix (Sec. "CPU Data Collation": the
 * correlator handles lost UDP packets from the stations and produces a
 * weighting matrix along with the visibilities; Sec. "Calibration
 * Pipeline", weighting: visibilities are re-weighted for the lost data).
 *
 * A spectrum s of antenna a is valid iff every input sample of its FIR
 * window, samples s*Ps .. (s+T)*Ps - 1 (Ps = 64 for afc_channelise, 256 for
 * afc_channelise_fine), arrived.  The masked chain is
 *   channelise -> afc_validity -> afc_zero_invalid -> afc_correlate
 *   -> afc_validity_weights [-> afc_normalise_visibilities]
 * so that V_ab sums the spectra valid for both antennas (zeroed samples add
 * exactly nothing) and W_ab counts them.
 *
 * afc_validity_words  uint32 words of the validity mask: B * ceil(S/32) * Na.
 * afc_validity   packet_valid uint8 [B][n_packets][Na], nonzero = packet k
 *                of antenna a arrived; a packet holds packet_samples
 *                consecutive input samples (sample n is in packet
 *                n / packet_samples; samples past the last packet count as
 *                lost).  spec_valid out: uint32 [B][ceil(S/32)][Na], bit
 *                s % 32 of word s / 32 set iff spectrum s is valid; bits of
 *                s >= S are 0.
 * afc_zero_invalid  sets to zero, in z (afc_channelise layout, type dt), the
 *                samples of both receivers of antenna a, in every channel,
 *                of each spectrum invalid for a.  Writes only those samples.
 * afc_validity_weights  weights int32 [B][Nbl]: the number of spectra
 *                s < S_b valid for both antennas (n_spectra_per_sb host
 *                [B] or NULL = all S), 0 when either is flagged (flags
 *                uint8 [B][Na] or NULL).  Use it in place of the weights of
 *                afc_correlate.
 * afc_normalise_visibilities  out float2 [B][P][Nbl][2][2] = vis / W per
 *                baseline (0 where W = 0): the mean visibility per valid
 *                spectrum.  vis is int2 for vis_dtype AFC_I8 (divided in
 *                float64, rounded once) and float2 otherwise (one float32
 *                division).  out may not alias vis.
 * ------------------------------------------------------------------------- */
AFC_API size_t afc_validity_words(const afc_dims* d);
AFC_API int afc_validity(const afc_dims* d, const uint8_t* packet_valid, int32_t n_packets,
                         int32_t packet_samples, int32_t samples_per_spectrum,
                         uint32_t* spec_valid, hipStream_t stream);
AFC_API int afc_zero_invalid(const afc_dims* d, afc_dtype dt, const uint32_t* spec_valid, void* z,
                             hipStream_t stream);
AFC_API int afc_validity_weights(const afc_dims* d, const uint32_t* spec_valid,
                                 const int32_t* n_spectra_per_sb, const uint8_t* flags,
                                 int32_t* weights, hipStream_t stream);
AFC_API int afc_normalise_visibilities(const afc_dims* d, afc_dtype vis_dtype, const void* vis,
                                       const int32_t* weights, void* out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * afc_calibrate_grad -- gain-calibration loss and its gradient
 * (Sec. "Calibration Pipeline": per-channel amplitude and phase calibration
 * of XX and YY against a point-source sky model; least-squares reading).
 * Per channel k and polarisation pol in {X, Y}:
 *
 *   R_ab = V_ab - g_a M_ab conj(g_b),   L = sum_{a,b} |R_ab|^2 (full matrix)
 *   grad_a = dL/dRe g_a + i dL/dIm g_a
 *          = -2 sum_b [ R_ab conj(M_ab) + conj(R_ba) M_ba ] g_b
 *
 * V, M     float2 [P][Nbl][2][2] lower triangles in the afc_correlate layout;
 *          the upper triangle is the conjugate.  XX = [0][0], YY = [1][1];
 *          XY, YX are not read.
 * g        float2 [P][Na][2]: gain of antenna a, polarisation pol.
 * loss     double [P][2] (XX, YY).  Residuals are evaluated in float32 with
 *          error-free product/sum transformations (no float64); the loss sum
 *          is float32, stored widened.
 * grad     float2 [P][Na][2], or NULL for the loss only.  Per-element terms
 *          in float32; the per-antenna sums are accumulated in float64.
 * workspace  device buffer of afc_calibrate_workspace_bytes(Na, P) bytes.
 * Limits: n_antennas <= 4096.
 * ------------------------------------------------------------------------- */
AFC_API size_t afc_calibrate_workspace_bytes(int32_t n_antennas, int32_t n_channels);
AFC_API int afc_calibrate_grad(int32_t n_antennas, int32_t n_channels, const void* V,
                               const void* M, const void* g, double* loss, void* grad,
                               void* workspace, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * afc_calibrate_grad_noalloc -- afc_calibrate_grad without a workspace, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * kernels and results as afc_calibrate_grad; it calls no allocator.
 *
 * The per-tile partial sums live in a fixed array of
 * AFC_CAL_NOALLOC_MAX_BYTES bytes of device memory that the library holds on
 * every GPU it runs on until the process ends (its address is looked up once
 * per device, on the first call there).  Shapes whose
 * afc_calibrate_workspace_bytes exceeds that size return AFC_ERR_UNSUPPORTED
 * (576 antennas x 64 channels need 11.8 MB).  Nothing in the array has to
 * start at zero, but all calls on one GPU share it: calls that overlap on
 * one GPU (two streams or two threads) race and must be serialised.
 * ------------------------------------------------------------------------- */
#define AFC_CAL_NOALLOC_MAX_BYTES (16u << 20)
AFC_API int afc_calibrate_grad_noalloc(int32_t n_antennas, int32_t n_channels, const void* V,
                                       const void* M, const void* g, double* loss, void* grad,
                                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * afc_calibrate_solve -- per-channel gains for XX and YY (Sec. "Calibration
 * Pipeline": amplitude and phase calibration at the channel level against
 * a point-source model), minimising the afc_calibrate_grad loss.
 *
 * n_iter iterations, every gain at once from the previous iterate:
 *   g_a <- g_a - grad_a / (4 D_a),   D_a = sum_b |M_ab|^2 |g_b|^2
 * with grad the afc_calibrate_grad gradient; since grad_a = -4 (sum_b V_ab
 * conj(z_ab) - g_a D_a), z_ab = M_ab conj(g_b), this is the least-squares
 * optimum of each g_a with the others fixed (the StEFCal iteration of
 * Salvini & Wijnholds, 2014).  On every second iteration the new iterate is
 * averaged with the previous one.  Gains with D_a = 0 stay unchanged.
 * Finally each (channel, polarisation) is rotated so that g_0 is real and
 * positive (the loss is blind to a common phase).
 *
 * V, M     as afc_calibrate_grad; flagged entries may be zeroed first
 *          (afc_apply_vis_flags): a zero V_ab with a zero M_ab drops out.
 * g        float2 [P][Na][2]: initial gains in, solution out.
 * loss     double [P][2] of the solution, or NULL.
 * workspace  afc_calibrate_solve_workspace_bytes(Na, P) bytes.
 * Limits: n_antennas <= 4096, 0 <= n_iter <= 100000.
 * ------------------------------------------------------------------------- */
AFC_API size_t afc_calibrate_solve_workspace_bytes(int32_t n_antennas, int32_t n_channels);
AFC_API int afc_calibrate_solve(int32_t n_antennas, int32_t n_channels, const void* V,
                                const void* M, void* g, int32_t n_iter, double* loss,
                                void* workspace, hipStream_t stream);

/* -------------------------------------------------------------------------
 * afc_calibrate_grad_weighted, afc_calibrate_solve_weighted -- the loss,
 * gradient and solver above on flagged and re-weighted visibilities
 * (Sec. "Real-time Flagging, Calibration and Imaging": lost packets re-weight
 * the visibilities, sigma clipping flags them, and calibration works on the
 * flagged visibilities).  With a real weight w_ab per stored baseline and
 * polarisation (w_ba = w_ab):
 *
 *   L = sum_{a,b} w_ab |R_ab|^2
 *   grad_a = -2 sum_b [ w_ab R_ab conj(M_ab) + w_ba conj(R_ba) M_ba ] g_b
 *   solver: D_a = sum_b w_ab |M_ab|^2 |g_b|^2 (the weighted least-squares
 *           optimum of each g_a with the others fixed)
 *
 * w_ab = 0 where vis_flags is nonzero, else weights[...] (or 1 when weights
 * is NULL).  Both arrays are [P][Nbl][2] (channel, baseline, XX / YY), the
 * layout afc_sigma_clip writes; either may be NULL (both NULL = the
 * unweighted entry points, bit for bit).  vis_flags must be 2-byte and
 * weights 8-byte aligned (AFC_ERR_INVALID otherwise).  Weights must be
 * finite and >= 0 (finiteness is checked in checked mode; the sign is not
 * checked).
 * All other arguments, the workspace sizes and the limits are those of
 * afc_calibrate_grad and afc_calibrate_solve.
 * ------------------------------------------------------------------------- */
AFC_API int afc_calibrate_grad_weighted(int32_t n_antennas, int32_t n_channels, const void* V,
                                        const void* M, const uint8_t* vis_flags,
                                        const float* weights, const void* g, double* loss,
                                        void* grad, void* workspace, hipStream_t stream);
AFC_API int afc_calibrate_solve_weighted(int32_t n_antennas, int32_t n_channels, const void* V,
                                         const void* M, const uint8_t* vis_flags,
                                         const float* weights, void* g, int32_t n_iter,
                                         double* loss, void* workspace, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * afc_sigma_clip -- real-time flagging (Sec. "Calibration Pipeline",
 * flagging: sigma clipping of visibility amplitudes against a threshold
 * above the locally computed RMS, first across the visibilities within a
 * channel, then across the channels of every visibility), on XX and YY:
 *   stage 1, per (channel, pol): RMS^2 = mean |V_ab|^2 over a != b;
 *            flag |V_ab| > threshold * RMS
 *   stage 2, per (baseline, pol): RMS^2 = mean |V_ab|^2 over the channels
 *            not flagged in stage 1; flag |V_ab| > threshold * RMS
 * Autocorrelations are neither used nor flagged.  |V|^2 in float64; sums in
 * a fixed order (reproducible).
 * V          float2 [P][Nbl][2][2] (the afc_correlate / afc_normalise layout).
 * vis_flags  uint8 [P][Nbl][2] out (XX, YY): 1 = flagged.
 * workspace  afc_sigma_clip_workspace_bytes(Na, P) bytes.
 *
 * afc_apply_vis_flags sets the flagged XX / YY entries of V and of M (either
 * may be NULL) to zero, in place.
 * ------------------------------------------------------------------------- */
AFC_API size_t afc_sigma_clip_workspace_bytes(int32_t n_antennas, int32_t n_channels);
AFC_API int afc_sigma_clip(int32_t n_antennas, int32_t n_channels, const void* V, float threshold,
                           uint8_t* vis_flags, void* workspace, hipStream_t stream);
AFC_API int afc_apply_vis_flags(int32_t n_antennas, int32_t n_channels, const uint8_t* vis_flags,
                                void* V, void* M, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Gridding and imaging (Sec. "Imaging Pipeline": the calibrated visibilities
 * of several subbands are gridded onto one common grid with bilinear
 * interpolation, which integrates them spectrally, and the grid is Fourier
 * transformed into the snapshot image: 1024 x 1024 pixels for AARTFAAC-6,
 * 2048 x 2048 for AARTFAAC-12).
 *
 * afc_grid_visibilities
 *   vis       float2 [B][64][Nbl][2][2] (afc_correlate / afc_normalise
 *             layout, calibrated); Stokes I = (XX + YY) / 2 is gridded.
 *   weights   int32 [B][Nbl] (natural weights, e.g. afc_validity_weights)
 *             or NULL (1); baselines of weight 0 are skipped.
 *   positions double [Na][2] east / north antenna positions in metres.
 *   freq_hz   double [B][64] sky frequency of every channel (device).
 *   For each cross-correlation a > c: u = (x_a - x_c) nu / c, v = (y_a -
 *   y_c) nu / c; (pu, pv) = (u, v) / cell_wavelengths + N/2; w I is spread
 *   bilinearly over the four cells around (pu, pv) and w conj(I) over the
 *   mirrored cells (N - j, N - i).  A visibility is gridded only if all
 *   eight cells lie inside the grid (1 <= floor(pu), floor(pv) <= N - 2).
 *   grid      float2 [N][N] out, indexed [v][u] (un-normalised sums).
 *   norm      double [1] out (device): sum of 2 w over gridded visibilities.
 *   The sums are formed in 64-bit fixed point with integer atomics, so the
 *   grid is bitwise reproducible run to run.
 * afc_image_from_grid
 *   image     float [N][N] out: image[j][i] = Re sum_{q,p} grid[q][p]
 *             exp(-2 pi i ((p - N/2)(i - N/2) + (q - N/2)(j - N/2)) / N)
 *             / norm; pixel (i, j) at l = (i - N/2) / (N du), m = (j - N/2)
 *             / (N du) (du = 1/2 wavelength images the whole sky).  A unit
 *             point source peaks near 1 at its pixel.  Float32 FFT.
 * workspace  afc_imaging_workspace_bytes(Na, B, N) bytes, shared by both.
 * Limits: N a power of two in 32..4096; n_antennas <= 4096.
 * ------------------------------------------------------------------------- */
AFC_API size_t afc_imaging_workspace_bytes(int32_t n_antennas, int32_t n_subbands, int32_t grid_size);
AFC_API int afc_grid_visibilities(int32_t n_antennas, int32_t n_subbands, const void* vis,
                                  const int32_t* weights, const double* positions,
                                  const double* freq_hz, int32_t grid_size, double cell_wavelengths,
                                  void* grid, double* norm, void* workspace, hipStream_t stream);
AFC_API int afc_image_from_grid(int32_t grid_size, const void* grid, const double* norm, float* image,
                                void* workspace, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batching form (Sec. "GPU Processing": each subband is an independent unit
 * of work; the paper hands subbands to free GPUs one by one, here all of them
 * go into one channeliser launch and one correlator launch per family of
 * sample types (int8 + fp16 together, fp32 apart) whose workgroups each take
 * one tile of a host-built, XCD-balanced work list, replayed as a HIP graph).
 *
 * afc_plan_create    d: shape with n_spectra = max S_b; dtype_per_sb host
 *                    [B] (AFC_F16 or AFC_I8 each, or AFC_F32); n_spectra_per_sb
 *                    host [B]; tune_cache_path: a JSON file of measured
 *                    choices {"key": [tile, workgroups per CU, split]} (read,
 *                    and written after tuning; split = 1 puts int8 and fp16
 *                    subbands in correlator launches of their own), or NULL
 *                    for the built-in default (128, 2, 0).  Tuning runs kernels on the current
 *                    device at creation time on scratch memory it allocates
 *                    and frees there.
 * afc_plan_workspace_bytes  bytes of the caller-owned workspace that holds
 *                    the channelised samples of all subbands (each subband in
 *                    its own type).
 * afc_plan_launch    x: int16 [B][L][N][2] with L = (n_spectra + T - 1) * P
 *                    (subband b reads its first (S_b + T - 1) * P rows);
 *                    gain_per_sb host float [B] (used for int8 subbands);
 *                    flags uint8 [B][Na] or NULL; vis [B][P][Nbl][2][2]
 *                    (float2 or int2 per subband type, 16-byte aligned);
 *                    weights int32 [B][Nbl]
 *                    or NULL.  A launch with new buffers or new gains
 *                    captures the work into a new HIP graph (allocating its
 *                    B * 32-byte item table, uploaded asynchronously on
 *                    `stream`); launches with the same buffers and gains only
 *                    enqueue that graph on `stream`.  A replaced graph and its
 *                    table stay alive until its last launch has completed
 *                    (an event recorded on the launch stream), and are freed
 *                    by a later call or by afc_plan_destroy, so launches
 *                    still in flight never see the new gains.  Freeing may
 *                    synchronise the device; plans are not thread-safe.
 * afc_plan_destroy   waits for the plan's graphs to finish, then frees them
 *                    and the plan.
 * ------------------------------------------------------------------------- */
typedef struct afc_plan afc_plan;

AFC_API int afc_plan_create(const afc_dims* d, const afc_dtype* dtype_per_sb,
                            const int32_t* n_spectra_per_sb, const char* tune_cache_path,
                            afc_plan** out);
AFC_API size_t afc_plan_workspace_bytes(const afc_plan* p);
AFC_API int afc_plan_launch(afc_plan* p, const int16_t* x, const float* taps,
                            const float* gain_per_sb, void* z_workspace,
                            const uint8_t* flags, void* vis, int32_t* weights,
                            hipStream_t stream);
/* Tile configuration the plan's correlator uses (host out-params):
 * tile width, workgroups of its launch and work items in the list. */
AFC_API int afc_plan_info(const afc_plan* p, int32_t* tile_rows, int32_t* tile_cols,
                          int32_t* n_workgroups, int32_t* n_work_items);
AFC_API void afc_plan_destroy(afc_plan* p);

/* ---------------------------------------------------------------------------
 * Checked (debug) mode.  With it on, every entry point first counts the
 * non-finite values (NaN, +-Inf) of its floating-point inputs on the device
 * and returns AFC_ERR_INVALID, naming the input and the count, if there are
 * any: taps, bandpass and delays of the channelisers, z of afc_correlate
 * (fp32 / fp16), vis of afc_normalise_visibilities (float), V, M and g of the
 * calibration calls, V of afc_sigma_clip, vis, positions and freq_hz of the
 * gridder, the grid of the imager.  A checked call reads the count back and
 * so waits for its stream: keep the mode off under graph capture and on the
 * hot path (it is off by default; the switch is process-wide).
 *
 * afc_count_nonfinite  the count behind it, for any device buffer of n
 *                      values of the given type; *count (host) is written
 *                      after the stream has passed the count.  The count
 *                      uses one device counter per GPU; counts from several
 *                      host threads run one after another.
 * ------------------------------------------------------------------------- */
typedef enum {
    AFC_VALUES_F32 = 0,
    AFC_VALUES_F16 = 1,
    AFC_VALUES_F64 = 3
} afc_value_type;
AFC_API void afc_set_checked_mode(int on);
AFC_API int afc_checked_mode(void);
AFC_API int afc_count_nonfinite(const void* values, size_t n, afc_value_type type, uint64_t* count,
                                hipStream_t stream);

/* Message for the last non-OK return on this thread ("" if none). */
AFC_API const char* afc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AFC_H */
