"""Benchmark of the FX-correlator hot path on one MI355X.

One step = one pass of the hot path over one integration of the AARTFAAC-12
shaped workload (576 dual-polarised antennas = 1152 receivers, 16 subbands,
64 channels, 3051 spectra ~ 1 s): afc_channelise (16-tap PPF, requantised to
int8) followed by afc_correlate (int8 MFMA X-engine, lower triangle).
Inputs are synthetic, seeded, and resident in HBM before timing starts.

Prints ONE JSON line.  `value` is the whole step's useful complex
multiply-accumulates per second (TCMAC/s).  Beside it: per-kernel times from
HIP events on the launch stream, the X-engine's fraction of the int8 MFMA
peak (and the MACs it issues including diagonal-tile and padding waste), the
PPF's algorithmic GB/s, the real-time factor, the lost-packet path on the
same step (validity masks, zeroing, weighting matrix, normalisation), the
fp32 path for the
int8-vs-fp32 comparison, the host-to-device rate of the int16 input (not in
the step), the whole 32-subband band of the same shape, the paper's
256-channel configuration (fused delay/bandpass compensation and 4:1 channel
integration, then the X-engine), the batching plan
(32 subbands, ragged, flagged, mixed fp16/int8), the calibration
gradient, gain solver and sigma-clip flagger, gridding and imaging of 8
subbands on a 2048^2 grid, and the CPU oracle timed on a
bounded sample on the host cores.
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "X-engine TCMAC/s and % MFMA peak, int8 vs fp32, 576 ant; PPF GB/s; real-time factor"
PEAK_HBM_GBS = 8000.0
PEAK_INT8_TOPS = 5000.0
PEAK_FP16_TFLOPS = 2500.0
PEAK_FP32_MFMA_TFLOPS = 157.3
# fp32 vector peak (datasheet): 256 CU x 4 SIMD x 16 lanes x 2 (packed fp32) x
# 2 flop (FMA) x 2.4 GHz = 157.3 TFLOP/s.  Without packed fp32 instructions,
# which this library does not use, a wave64 FMA takes 4 cycles: 78.6 TFLOP/s
# (a plain FMA loop measures 74.5 TFLOP/s).
PEAK_FP32_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel_key):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by a plain 1 GiB copy), or
    None when the kernel's sources (its .hip file and the headers it shares)
    have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        d = json.load(open(path))
        k = d["kernels"][kernel_key]
        h = hashlib.sha256()
        for f in k["sources"]:
            h.update(open(os.path.join(ROOT, "paper_1609_04205_amd", "csrc", f), "rb").read())
        if h.hexdigest()[:16] != k["sources_sha256_16"]:
            return None
        return round(k["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="time only the int8 step")
    ap.add_argument("--cpu-sample-spectra", type=int, default=3051)
    ap.add_argument("--cpu-one-thread-spectra", type=int, default=64)
    ap.add_argument("--fine-only", action="store_true",
                    help="only time the 256-channel configuration (fine channeliser + X-engine on its output)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (three times), to scale HBM byte counters")
    return ap.parse_args()


class Timer:
    """Average kernel durations from HIP events recorded on the launch stream."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def rec(self, name):
        torch = self.torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        self.pairs.setdefault(name, []).append((e0, e1))
        return e1

    def ms(self, name):
        ps = self.pairs.get(name, [])
        return sum(a.elapsed_time(b) for a, b in ps) / max(1, len(ps))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        a = torch.ones((1 << 30) // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}), flush=True)
        return

    import paper_1609_04205_amd as afc
    import workloads as W

    dev = torch.device("cuda:0")
    cfg = W.A12
    if args.fine_only:
        print(json.dumps({"fine": run_fine(torch, afc, W, dev, cfg, reps=args.steps)}), flush=True)
        return
    B, Na, S, P = cfg.n_subbands, cfg.n_antennas, cfg.n_spectra, 64
    N = 2 * Na
    nbl = Na * (Na + 1) // 2
    L = cfg.n_rows
    log(f"workload {cfg.name}: B={B} Na={Na} N={N} S={S}")
    x = W.make_voltages(cfg, device=dev)
    taps_np = W.prototype_taps()
    taps = torch.from_numpy(taps_np).to(dev)
    gain = W.requant_gain(cfg, taps_np)
    z8 = torch.empty(afc.channelised_shape(B, S, N), dtype=torch.int8, device=dev)
    vis = torch.empty(afc.visibility_shape(B, Na), dtype=torch.int32, device=dev)
    wts = torch.empty((B, nbl), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    timer = Timer(torch)

    def step(tm=None):
        if tm:
            e = tm.rec("ppf")
        afc.channelise(x, taps, S, "i8", gain, out=z8)
        if tm:
            e.record(torch.cuda.current_stream())
            e = tm.rec("xengine")
        afc.correlate(z8, n_spectra=S, out=vis, weights=wts)
        if tm:
            e.record(torch.cuda.current_stream())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timer)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    ppf_ms, xe_ms = timer.ms("ppf"), timer.ms("xengine")

    cmac = float(B) * P * (N * (N + 1) // 2) * S             # useful complex MACs per step
    data_s = S * P / W.F_SUBBAND                              # seconds of data per step
    ppf_bytes = float(B) * L * N * 4 + float(B) * P * S * N * 2 + 4 * 16 * 64
    # FIR 16 taps x 4 flop per complex point + FFT 5 log2(64) flop per point
    ppf_flops = float(B) * N * S * 64 * (16 * 4 + 5 * 6)
    xe_tops = 8.0 * cmac / (xe_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(cmac / (ms_step * 1e-3) / 1e12, 4),
        "unit": "TCMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "a12-576ant-16sb-3051spectra", "n_antennas": Na, "n_receivers": N,
                   "n_subbands": B, "n_channels": P, "n_taps": 16, "n_spectra": S,
                   "step": "channelise(int16 -> int8) + correlate(int8 MFMA, int32)"},
        "roofline": None,
        "real_time_factor": round(data_s / (ms_step * 1e-3), 2),
        "xengine_ms": round(xe_ms, 4),
        "xengine_tcmacs": round(cmac / (xe_ms * 1e-3) / 1e12, 3),
        "xengine_int8_mfma_frac": round(xe_tops / PEAK_INT8_TOPS, 4),
        "ppf_ms": round(ppf_ms, 4),
        "ppf_gbs": round(ppf_bytes / (ppf_ms * 1e-3) / 1e9, 1),
        "ppf_hbm_frac": round(ppf_bytes / (ppf_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "ppf_valu_frac": round(ppf_flops / (ppf_ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
    }
    ppf_roof = {"bound": "hbm", "achieved": round(ppf_bytes / (ppf_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(ppf_bytes / (ppf_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic("ppf_kernel<int8>")}
    xe_roof = {"bound": "mfma", "achieved": round(xe_tops, 2), "peak": PEAK_INT8_TOPS, "unit": "TFLOP/s",
               "frac": round(xe_tops / PEAK_INT8_TOPS, 4), "traffic": measured_traffic("xengine_kernel<int8,128>")}
    out["roofline"] = xe_roof if xe_ms >= ppf_ms else ppf_roof
    out["roofline_other"] = ppf_roof if xe_ms >= ppf_ms else xe_roof
    # complex MACs the int8 X-engine actually issues on MFMA: whole 128 x 128
    # off-diagonal tiles, 36 of the 64 16 x 16 blocks per diagonal tile;
    # spectra padded to whole stages of 4 blocks of 8, and off the diagonal
    # the stage count to a multiple of the 3-stage register ring
    T = -(-N // 128)
    nb = (S + 7) // 8
    spectra_off = -(-nb // 12) * 12 * 8
    spectra_diag = -(-nb // 4) * 4 * 8
    computed = float(B) * P * (T * (T - 1) // 2 * 128 * 128 * spectra_off + T * 36 * 16 * 16 * spectra_diag)
    out["xengine_computed_cmac"] = computed
    out["xengine_useful_fraction"] = round(cmac / computed, 4)
    log(f"int8 step {ms_step:.3f} ms (ppf {ppf_ms:.3f}, xengine {xe_ms:.3f})")

    if not args.no_extras:
        # ---- lost packets on the same step: validity masks from packet flags
        # (0.1% of the packets lost in bursts, one station dead in one
        # subband), zeroing of invalid spectra, the weighting matrix, and the
        # visibilities divided by their weights
        pkt_np = W.packet_loss(B, Na, L, seed=cfg.seed, dead=[(5, 7)])
        pkt = torch.from_numpy(pkt_np).to(dev)
        bits = torch.empty(afc.validity_shape(B, S, Na), dtype=torch.int32, device=dev)
        visn = torch.empty(vis.shape, dtype=torch.float32, device=dev)
        tv = Timer(torch)
        for it in range(4):
            tm = tv if it > 0 else None
            for name, fn in (("validity", lambda: afc.validity(pkt, S, W.PACKET_SAMPLES, out=bits)),
                             ("zero", lambda: afc.zero_invalid(z8, bits, S)),
                             ("weights", lambda: afc.validity_weights(bits, S, out=wts)),
                             ("normalise", lambda: afc.normalise_visibilities(vis, wts, out=visn))):
                e = tm.rec(name) if tm else None
                fn()
                if e is not None:
                    e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms_v = {k: tv.ms(k) for k in ("validity", "zero", "weights", "normalise")}
        norm_bytes = 2.0 * vis.numel() * 4 + wts.numel() * 4
        out["lost_packets"] = {"packets_lost_fraction": round(1.0 - float(pkt_np.mean()), 5),
                               "validity_ms": round(ms_v["validity"], 4), "zero_invalid_ms": round(ms_v["zero"], 4),
                               "weights_ms": round(ms_v["weights"], 4),
                               "masked_step_overhead": round((ms_v["validity"] + ms_v["zero"] + ms_v["weights"])
                                                             / ms_step, 4),
                               "normalise_ms": round(ms_v["normalise"], 3),
                               "normalise_gbs": round(norm_bytes / (ms_v["normalise"] * 1e-3) / 1e9, 1)}
        log(f"lost packets: validity {ms_v['validity']:.3f} zero {ms_v['zero']:.3f} weights {ms_v['weights']:.3f} "
            f"normalise {ms_v['normalise']:.3f} ms")
        del pkt, bits, visn

        # ---- the same int8 X-engine launch on all-zero samples: the cycles
        # are the same, the shader clock is not (the MFMAs draw less power
        # on constant operand data), so this is the kernel at a clock the
        # chip sustains only for such data
        z8.zero_()
        tzr = Timer(torch)
        for it in range(3):
            e = tzr.rec("xengine") if it > 0 else None
            afc.correlate(z8, n_spectra=S, out=vis, weights=wts)
            if e is not None:
                e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        out["xengine_int8_zero_samples_ms"] = round(tzr.ms("xengine"), 3)
        log(f"int8 xengine on zero samples {tzr.ms('xengine'):.3f} ms")

        # ---- fp32 path on the same input: int8 vs fp32
        del z8
        z32 = torch.empty(afc.channelised_shape(B, S, N), dtype=torch.float32, device=dev)
        vis32 = torch.empty(afc.visibility_shape(B, Na), dtype=torch.float32, device=dev)
        t32 = Timer(torch)
        for it in range(3):
            tm = t32 if it > 0 else None
            if tm:
                e = tm.rec("ppf")
            afc.channelise(x, taps, S, "f32", out=z32)
            if tm:
                e.record(torch.cuda.current_stream())
                e = tm.rec("xengine")
            afc.correlate(z32, n_spectra=S, out=vis32, weights=wts)
            if tm:
                e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        f32_xe = t32.ms("xengine")
        f32_tf = 8.0 * cmac / (f32_xe * 1e-3) / 1e12
        out["fp32"] = {"xengine_ms": round(f32_xe, 3), "xengine_tcmacs": round(cmac / (f32_xe * 1e-3) / 1e12, 3),
                       "xengine_fp32_mfma_frac": round(f32_tf / PEAK_FP32_MFMA_TFLOPS, 4),
                       "ppf_ms": round(t32.ms("ppf"), 3),
                       "ppf_gbs": round((float(B) * L * N * 4 + float(B) * P * S * N * 8) / (t32.ms("ppf") * 1e-3) / 1e9, 1),
                       "real_time_factor": round(data_s / ((f32_xe + t32.ms("ppf")) * 1e-3), 2)}
        out["int8_speedup_over_fp32_xengine"] = round(f32_xe / xe_ms, 2)
        log(f"fp32 xengine {f32_xe:.3f} ms")
        parity_vis = {"f32": _sampled_vis(torch, vis32, 0, PARITY_ANTENNAS)}
        del z32, vis32

        # ---- fp16 path on the same input (fp16 samples, float32 accumulation)
        z16 = torch.empty(afc.channelised_shape(B, S, N), dtype=torch.float16, device=dev)
        vis16 = torch.empty(afc.visibility_shape(B, Na), dtype=torch.float32, device=dev)
        t16 = Timer(torch)
        for it in range(3):
            tm = t16 if it > 0 else None
            if tm:
                e = tm.rec("ppf")
            afc.channelise(x, taps, S, "f16", out=z16)
            if tm:
                e.record(torch.cuda.current_stream())
                e = tm.rec("xengine")
            afc.correlate(z16, n_spectra=S, out=vis16, weights=wts)
            if tm:
                e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        f16_xe = t16.ms("xengine")
        f16_tf = 8.0 * cmac / (f16_xe * 1e-3) / 1e12
        out["fp16"] = {"xengine_ms": round(f16_xe, 3), "xengine_tcmacs": round(cmac / (f16_xe * 1e-3) / 1e12, 3),
                       "xengine_fp16_mfma_frac": round(f16_tf / PEAK_FP16_TFLOPS, 4),
                       "ppf_ms": round(t16.ms("ppf"), 3),
                       "ppf_gbs": round((float(B) * L * N * 4 + float(B) * P * S * N * 4) / (t16.ms("ppf") * 1e-3) / 1e9, 1),
                       "real_time_factor": round(data_s / ((f16_xe + t16.ms("ppf")) * 1e-3), 2)}
        log(f"fp16 xengine {f16_xe:.3f} ms")
        parity_vis["f16"] = _sampled_vis(torch, vis16, 0, PARITY_ANTENNAS)
        parity_x0 = x[0].cpu().numpy()
        del z16, vis16, x, vis
        torch.cuda.empty_cache()

        # ---- host-to-device copy of the int16 input (not part of the step:
        # the entry points take device buffers), one subband-second at a time
        xh = torch.empty((L, N, 2), dtype=torch.int16, pin_memory=True)
        xd = torch.empty((L, N, 2), dtype=torch.int16, device=dev)
        th = Timer(torch)
        for it in range(4):
            e = th.rec("h2d") if it > 0 else None
            xd.copy_(xh, non_blocking=True)
            if e is not None:
                e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        h2d_ms = th.ms("h2d")
        sb_bytes = float(L) * N * 4
        out["h2d"] = {"bytes_per_subband_second": sb_bytes, "gbs": round(sb_bytes / (h2d_ms * 1e-3) / 1e9, 1),
                      "ms_per_subband_second": round(h2d_ms, 3),
                      "step_ms_with_h2d": round(ms_step + B * h2d_ms, 3),
                      "real_time_factor_with_h2d": round(data_s / ((ms_step + B * h2d_ms) * 1e-3), 2)}
        log(f"h2d {h2d_ms:.3f} ms per subband-second")
        del xh, xd

        # ---- the whole AARTFAAC-12 band: 32 subbands of the same shape
        cfg_band = W.Config("a12-576ant-32sb", Na, 32, n_spectra=S, sigma_n=cfg.sigma_n, n_sources=cfg.n_sources,
                         seed=cfg.seed, layout=cfg.layout)
        x_band = W.make_voltages(cfg_band, device=dev)
        z32b = torch.empty(afc.channelised_shape(32, S, N), dtype=torch.int8, device=dev)
        v32 = torch.empty(afc.visibility_shape(32, Na), dtype=torch.int32, device=dev)
        w32 = torch.empty((32, nbl), dtype=torch.int32, device=dev)
        t32b = Timer(torch)
        for it in range(3):
            e = t32b.rec("step") if it > 0 else None
            afc.channelise(x_band, taps, S, "i8", gain, out=z32b)
            afc.correlate(z32b, n_spectra=S, out=v32, weights=w32)
            if e is not None:
                e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms32 = t32b.ms("step")
        out["a12_32sb"] = {"ms": round(ms32, 3), "tcmacs": round(2 * cmac / (ms32 * 1e-3) / 1e12, 3),
                           "real_time_factor": round(data_s / (ms32 * 1e-3), 2)}
        log(f"32 subbands {ms32:.3f} ms")
        del x_band, z32b, v32, w32
        torch.cuda.empty_cache()

        # ---- the paper's channeliser configuration on the same array
        out["fine"] = run_fine(torch, afc, W, dev, cfg)

        # ---- batching form: 32 subbands, ragged S, flags, mixed fp16/int8, one graph
        cfgb = W.A12_BATCHED
        bp = W.batch_params(cfgb)
        dts = ["f16" if d == 1 else "i8" for d in bp.dtypes]
        xbat = W.make_voltages(cfgb, device=dev)
        tune_dir = tempfile.mkdtemp(prefix="afc_tune_")             # tuned afresh every run
        plan = afc.Plan(Na, bp.n_spectra.tolist(), dts, n_spectra=cfgb.n_spectra,
                        tune_cache=os.path.join(tune_dir, "tune_cache.json"))
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        visb = torch.empty(afc.visibility_shape(cfgb.n_subbands, Na), dtype=torch.int32, device=dev)
        wb = torch.empty((cfgb.n_subbands, nbl), dtype=torch.int32, device=dev)
        fl = torch.from_numpy(bp.flags).to(dev)
        gb = [W.requant_gain(cfgb, taps_np)] * cfgb.n_subbands
        plan.launch(xbat, taps, gb, ws, visb, flags=fl, weights=wb)
        torch.cuda.synchronize()
        tp = Timer(torch)
        for _ in range(3):
            e = tp.rec("plan")
            plan.launch(xbat, taps, gb, ws, visb, flags=fl, weights=wb)
            e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        nprime = [2 * (Na - int(bp.flags[b].sum())) for b in range(cfgb.n_subbands)]
        cm4 = sum(P * n * (n + 1) // 2 * int(bp.n_spectra[b]) for b, n in enumerate(nprime))
        plan_ms = tp.ms("plan")
        info = plan.info()
        try:
            choice = list(json.load(open(os.path.join(tune_dir, "tune_cache.json"))).values())[0]
        except (OSError, ValueError, IndexError):
            choice = None
        out["batching"] = {"workload": cfgb.name, "graph_ms": round(plan_ms, 3),
                           "useful_tcmacs": round(cm4 / (plan_ms * 1e-3) / 1e12, 3),
                           "real_time_factor": round(max(bp.n_spectra) * P / W.F_SUBBAND / (plan_ms * 1e-3), 2),
                           "flagged_antenna_fraction": round(float(bp.flags.mean()), 4),
                           "tuned": None if choice is None else {"tile": choice[0], "workgroups_per_cu": choice[1],
                                                                 "int8_fp16_split": bool(choice[2])},
                           "tile": info.tile, "workgroups": info.n_workgroups, "work_items": info.n_work_items}
        log(f"plan {plan_ms:.3f} ms")
        plan.close()
        del ws
        # the same work as two graphs, one per sample type: parts against the whole
        parts = {}
        for t in ("i8", "f16"):
            idx = [b for b in range(cfgb.n_subbands) if dts[b] == t]
            if not idx:
                continue
            sel = torch.as_tensor(idx, device=dev)
            xs = xbat.index_select(0, sel)
            pl = afc.Plan(Na, [int(bp.n_spectra[b]) for b in idx], [t] * len(idx), n_spectra=cfgb.n_spectra,
                          tune_cache=os.path.join(tune_dir, f"tune_{t}.json"))
            wss = torch.empty(pl.workspace_bytes, dtype=torch.uint8, device=dev)
            vs = torch.empty(afc.visibility_shape(len(idx), Na), dtype=torch.int32, device=dev)
            wsb = torch.empty((len(idx), nbl), dtype=torch.int32, device=dev)
            fs = fl.index_select(0, sel)
            gs = [gb[b] for b in idx]
            pl.launch(xs, taps, gs, wss, vs, flags=fs, weights=wsb)
            torch.cuda.synchronize()
            tt = Timer(torch)
            for _ in range(3):
                e = tt.rec("g")
                pl.launch(xs, taps, gs, wss, vs, flags=fs, weights=wsb)
                e.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            parts[t] = {"subbands": len(idx), "graph_ms": round(tt.ms("g"), 3)}
            pl.close()
            del xs, wss, vs, wsb
            torch.cuda.empty_cache()
        out["batching"]["per_type_graphs"] = parts
        out["batching"]["sum_of_parts_ms"] = round(sum(v["graph_ms"] for v in parts.values()), 3)
        log(f"plan parts {parts}")
        del xbat, visb, wb
        torch.cuda.empty_cache()

        # ---- calibration adjoint, 576 antennas x 64 channels
        Vc, Mc, gc = W.make_calibration(Na=576, P=64, seed=5)
        Vt, Mt, gt = (torch.from_numpy(a).to(dev) for a in (Vc, Mc, gc))
        wcal = torch.empty(afc._lib.afc_calibrate_workspace_bytes(576, 64), dtype=torch.uint8, device=dev)
        afc.calibrate_grad(Vt, Mt, gt, workspace=wcal)
        torch.cuda.synchronize()
        # 20 calls back to back between one pair of events (a call is ~0.16
        # ms of GPU work, so host launch gaps would otherwise be timed too)
        n_cal = 20
        tc = Timer(torch)
        e = tc.rec("cal")
        for _ in range(n_cal):
            afc.calibrate_grad(Vt, Mt, gt, workspace=wcal)
        e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        cal_ms = tc.ms("cal") / n_cal
        # V and M arrive in the correlator's [P][Nbl][2][2] layout: the
        # algorithmic bytes are both arrays (32 B per baseline each; the
        # hardware reads whole records), of which XX and YY are half
        cal_bytes = 2.0 * 64 * nbl * 4 * 8
        out["calibration"] = {"ms": round(cal_ms, 4), "algorithmic_gbs": round(cal_bytes / (cal_ms * 1e-3) / 1e9, 1),
                              "hbm_frac": round(cal_bytes / (cal_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                              "xx_yy_gbs": round(cal_bytes / 2 / (cal_ms * 1e-3) / 1e9, 1)}
        # the weighted gradient (sigma-clip flags and lost-data weights)
        nbl_c = 576 * 577 // 2
        flc = (torch.rand((64, nbl_c, 2), device=dev) < 0.05).to(torch.uint8)
        wtc = torch.rand((64, nbl_c, 2), device=dev) + 0.5
        afc.calibrate_grad(Vt, Mt, gt, workspace=wcal, flags=flc, weights=wtc)
        torch.cuda.synchronize()
        tcw = Timer(torch)
        e = tcw.rec("calw")
        for _ in range(n_cal):
            afc.calibrate_grad(Vt, Mt, gt, workspace=wcal, flags=flc, weights=wtc)
        e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        out["calibration"]["weighted_ms"] = round(tcw.ms("calw") / n_cal, 4)
        del wcal, flc, wtc
        log(f"calibration {cal_ms:.3f} ms")
        # ---- gain solver (30 iterations from unit gains) and sigma-clip flagging
        n_it = 30
        g_unit = torch.zeros_like(gt)
        g_unit[..., 0] = 1.0
        gs = g_unit.clone()
        wss = torch.empty(afc._lib.afc_calibrate_solve_workspace_bytes(576, 64), dtype=torch.uint8, device=dev)
        afc.calibrate_solve(Vt, Mt, gs, n_it, workspace=wss)
        flg = afc.sigma_clip(Vt, 5.0)
        torch.cuda.synchronize()
        ts = Timer(torch)
        for _ in range(3):
            gs.copy_(g_unit)
            e = ts.rec("solve")
            afc.calibrate_solve(Vt, Mt, gs, n_it, workspace=wss)
            e.record(torch.cuda.current_stream())
            e = ts.rec("clip")
            afc.sigma_clip(Vt, 5.0, out=flg)
            e.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        gsn = gs.cpu().numpy()
        gtn = gc[..., 0].astype(np.float64) + 1j * gc[..., 1]
        gtn = gtn * (np.conj(gtn[:, :1, :]) / np.abs(gtn[:, :1, :]))
        dev_true = float(np.abs((gsn[..., 0] + 1j * gsn[..., 1]) - gtn).max() / np.abs(gtn).max())
        out["calibration"].update({"solve_iterations": n_it, "solve_ms": round(ts.ms("solve"), 3),
                                   "solve_ms_per_iteration": round(ts.ms("solve") / n_it, 4),
                                   "solve_max_gain_error_vs_true": round(dev_true, 5),
                                   "sigma_clip_ms": round(ts.ms("clip"), 4)})
        log(f"solve {ts.ms('solve'):.3f} ms ({n_it} iterations), sigma clip {ts.ms('clip'):.3f} ms")
        del Vt, Mt, gt, gs, wss, flg
        torch.cuda.empty_cache()

        # ---- imaging: 8 subbands x 64 channels of the AARTFAAC-12 array
        # gridded onto 2048 x 2048 cells of half a wavelength, then the image
        out["imaging"] = run_imaging(torch, afc, W, dev, cfg)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_spectra, args.cpu_one_thread_spectra)
        if not args.no_extras:
            out["chain_error_vs_fp64"] = chain_error(parity_x0, parity_vis)
    print(json.dumps(out), flush=True)


def run_fine(torch, afc, W, dev, cfg, reps=3):
    """The paper's channeliser configuration on the given array: 256-channel
    bank, cable-delay and bandpass compensation, 4:1 channel integration (one
    fused kernel after a small table kernel), then the int8 X-engine on its
    output; about 1 s of data (762 spectra of 256 samples)."""
    B, Na, S, P = cfg.n_subbands, cfg.n_antennas, cfg.n_spectra, 64
    N = 2 * Na
    nbl = Na * (Na + 1) // 2
    Sf = S // 4                                               # 762 spectra of 256 samples
    xf = W.make_voltages(cfg, device=dev, n_rows=W.fine_rows(Sf))
    tf_np = W.prototype_taps(256, 16)
    bp_np = W.bandpass_weights()
    tapsf = torch.from_numpy(tf_np).to(dev)
    tau = torch.from_numpy(W.cable_delays(N)).to(dev)
    bpw = torch.from_numpy(bp_np).to(dev)
    nus = [W.subband_frequency(b) for b in range(B)]
    gf = W.fine_requant_gain(cfg, tf_np, bp_np)
    wsf = torch.empty(afc.fine_workspace_bytes(Na, B, Sf), dtype=torch.uint8, device=dev)
    zf = torch.empty(afc.channelised_shape(B, Sf, N), dtype=torch.int8, device=dev)
    visf = torch.empty(afc.visibility_shape(B, Na), dtype=torch.int32, device=dev)
    wf = torch.empty((B, nbl), dtype=torch.int32, device=dev)
    tfn = Timer(torch)
    for it in range(reps + 1):
        tm = tfn if it > 0 else None
        if tm:
            e = tm.rec("fine")
        afc.channelise_fine(xf, tapsf, Sf, tau, bpw, nus, W.F_SUBBAND, "i8", gf, out=zf, workspace=wsf)
        if tm:
            e.record(torch.cuda.current_stream())
            e = tm.rec("xengine")
        afc.correlate(zf, n_spectra=Sf, out=visf, weights=wf)
        if tm:
            e.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    f_ms, fx_ms = tfn.ms("fine"), tfn.ms("xengine")
    Lf = W.fine_rows(Sf)
    # int16 input, int8 output, the tables written once and read once, the taps
    fine_bytes = (float(B) * Lf * N * 4 + float(B) * P * ((Sf + 7) // 8) * 8 * N * 2
                  + (256 + N * 256 + B * N) * 8 * 2 + 16 * 256 * 4)
    cmac_f = float(B) * P * (N * (N + 1) // 2) * Sf
    data_f = Sf * 256 / W.F_SUBBAND
    res = {"workload": f"a12-576ant-16sb-{Sf}spectra-256ch-4to1",
                   "channelise_ms": round(f_ms, 3),
                   "channelise_gbs": round(fine_bytes / (f_ms * 1e-3) / 1e9, 1),
                   "channelise_hbm_frac": round(fine_bytes / (f_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                   "algorithmic_bytes": fine_bytes,
                   "channelise_ms_per_subband_second": round(f_ms / B / data_f, 3),
                   "xengine_ms": round(fx_ms, 3),
                   "step_ms": round(f_ms + fx_ms, 3),
                   "tcmacs": round(cmac_f / ((f_ms + fx_ms) * 1e-3) / 1e12, 3),
                   "real_time_factor": round(data_f / ((f_ms + fx_ms) * 1e-3), 2),
                   "traffic": measured_traffic("ppf_fine_kernel<int8>")}
    log(f"fine channeliser {f_ms:.3f} ms, xengine on its output {fx_ms:.3f} ms")
    del xf, zf, visf, wf, wsf
    torch.cuda.empty_cache()
    return res


def run_imaging(torch, afc, W, dev, cfg, B_img=8, N=2048, reps=3):
    """Gridding of B_img subbands (calibrated visibilities of three point
    sources, unit weights) and the 2-D FFT image of the AARTFAAC-12 array."""
    import numpy as np
    Na = cfg.n_antennas
    pos = torch.from_numpy(W.antenna_positions(cfg)).to(dev)
    freq = torch.tensor([[W.subband_frequency(b) + W.channel_offset(k, 64) * W.F_SUBBAND / 64 for k in range(64)]
                         for b in range(B_img)], dtype=torch.float64, device=dev)
    a, c = np.tril_indices(Na)
    dx, dy = pos[a, 0] - pos[c, 0], pos[a, 1] - pos[c, 1]
    vis = torch.zeros((B_img, 64, a.size, 2, 2, 2), dtype=torch.float32, device=dev)
    for flux, l0, m0 in ((10.0, 0.27, -0.31), (4.0, -0.12, 0.46), (2.0, 0.0, 0.07)):
        ph = 2.0 * np.pi / 299792458.0 * (dx[None, None, :] * l0 + dy[None, None, :] * m0) * freq[:, :, None]
        for p in range(2):
            vis[:, :, :, p, p, 0] += (flux * torch.cos(ph)).float()
            vis[:, :, :, p, p, 1] += (flux * torch.sin(ph)).float()
    del ph
    im = afc.Imager(pos, B_img, N, 0.5)
    grid = im.grid(vis, freq)
    img = im.image(grid)
    torch.cuda.synchronize()
    tm = Timer(torch)
    for _ in range(reps):
        e = tm.rec("grid")
        im.grid(vis, freq, out=grid)
        e.record(torch.cuda.current_stream())
        e = tm.rec("image")
        im.image(grid, out=img)
        e.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    n_vis = B_img * 64 * (Na * (Na - 1) // 2)
    res = {"workload": f"a12-576ant-{B_img}sb-grid{N}", "visibilities": n_vis,
           "grid_ms": round(tm.ms("grid"), 3),
           "grid_gvis_per_s": round(n_vis / (tm.ms("grid") * 1e-3) / 1e9, 2),
           "grid_vis_gbs": round(float(vis.numel()) * 4 / (tm.ms("grid") * 1e-3) / 1e9, 1),
           "image_ms": round(tm.ms("image"), 3)}
    log(f"imaging: grid {tm.ms('grid'):.3f} ms, image {tm.ms('image'):.3f} ms")
    del vis, grid, img, im
    torch.cuda.empty_cache()
    return res


# antennas whose baselines the chain-error comparison samples (subband 0, all channels)
PARITY_ANTENNAS = [0, 1, 47, 48, 95, 150, 199, 240, 287, 288, 333, 400, 431, 480, 529, 575]


def _sampled_vis(torch, vis, sb, ants):
    """Visibilities of the baselines among `ants` (a >= b) of subband sb, all
    channels, as complex128 numpy [P][n][2][2]."""
    bls = [a * (a + 1) // 2 + b for ia, a in enumerate(ants) for b in ants[: ia + 1]]
    v = vis[sb][:, torch.as_tensor(bls, device=vis.device)].double().cpu().numpy()
    return v[..., 0] + 1j * v[..., 1]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chain_int(x, S_s, threads):
    """Oracle chain of one subband (float64 PPF -> requant -> exact integer
    correlator over all 64 channels) on the first S_s spectra; returns the
    seconds of each stage and the useful CMACs."""
    import numpy as np

    import oracle
    import workloads as W

    cfg = W.A12
    N = cfg.n_inputs
    taps = W.prototype_taps()
    gain = W.requant_gain(cfg, taps)
    xs = np.ascontiguousarray(x[: (S_s + 15) * 64])
    t0 = time.perf_counter()
    y = oracle.ppf_subband(xs, taps, 64, 16, S_s)                         # [P][S][N]
    t1 = time.perf_counter()
    q = oracle.requant(np.stack([y.real, y.imag], -1).astype(np.float32), gain)
    t2 = time.perf_counter()
    for ch in range(64):
        oracle.xcorr_int(np.ascontiguousarray(q[ch]))
    t3 = time.perf_counter()
    return {"ppf_s": t1 - t0, "requant_s": t2 - t1, "correlator_s": t3 - t2, "total_s": t3 - t0,
            "cmac": 64.0 * (N * (N + 1) // 2) * S_s, "threads": threads}


def _one_thread_child(S_s, n_ch):
    """Entry of the child process that times the oracle on one thread (the
    OpenMP thread count is fixed when the oracle library loads); it never
    touches the GPU.  The channeliser and requantiser run on the first S_s
    spectra of all receivers; the correlator on n_ch channels of 3051 int8
    spectra (the same working set per channel as the full sample; its cost
    does not depend on the values).  Both are scaled to the full sample."""
    import numpy as np

    import oracle
    import workloads as W

    N = W.A12.n_inputs
    x = W.make_voltages(W.A12, subbands=[0], n_rows=(S_s + 15) * 64).numpy()[0]
    r = _oracle_chain_int(x, S_s, 1)
    q = np.random.default_rng(1).integers(-127, 128, size=(3051, N, 2)).astype(np.int8)
    t0 = time.perf_counter()
    for _ in range(n_ch):
        oracle.xcorr_int(q)
    t1 = time.perf_counter()
    full = (r["ppf_s"] + r["requant_s"]) * 3051 / S_s + (t1 - t0) * 64 / n_ch
    print(json.dumps({"full_sample_s": full, "ppf_requant_s": r["ppf_s"] + r["requant_s"], "corr_s": t1 - t0,
                      "cmac": 64.0 * (N * (N + 1) // 2) * 3051}), flush=True)


def cpu_baseline(S_s, S_1):
    """The oracle timed on the host cores, on bounded samples of the same
    workload and on two whole small configurations:
      value         oracle chain (float64 PPF -> requant -> exact-integer
                    correlator) of subband 0 of the AARTFAAC-12 workload, all
                    1152 receivers, the first S_s spectra, all 64 channels,
                    every host thread; TCMAC/s = useful CMACs / wall time
      one_thread    the same chain on the first S_1 spectra on one thread
      small_whole   the whole 48-antenna configuration (float64 PPF + float64
                    correlator, 3.05e8 CMAC)
      calibration_whole  the loss and gradient of 576 antennas x 64 channels
                    (XX, YY) at the true gains and at unit gains
    The input is drawn on the host with the same generator recipe (the
    device's draws differ); the oracle's cost does not depend on the values."""
    import numpy as np

    import oracle
    import workloads as W

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    x = W.make_voltages(W.A12, subbands=[0], n_rows=(S_s + 15) * 64).numpy()[0]
    main = _oracle_chain_int(x, S_s, threads)
    del x
    full_s = main["total_s"] * (3051 / S_s) * W.A12.n_subbands
    res = {"value": round(main["cmac"] / main["total_s"] / 1e12, 6), "unit": "TCMAC/s", "cores": threads,
           "kind": "oracle", "cpu_model": _cpu_model(),
           "sample": f"subband 0 of the AARTFAAC-12 workload, all {W.A12.n_inputs} receivers, first {S_s} of 3051 "
                     f"spectra, 64 channels: float64 PPF {main['ppf_s']:.1f} s + requant {main['requant_s']:.1f} s "
                     f"+ exact-int correlator {main['correlator_s']:.1f} s on {threads} threads",
           "workload_seconds_extrapolated": round(full_s, 1),
           "extrapolation": "linear in spectra and subbands to the 16-subband, 3051-spectrum step"}
    # one thread, in a child process (no GPU there), scaled to the 3051-spectrum sample
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-thread", str(S_1), "2"], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode == 0 and S_s == 3051:
        one = json.loads(r.stdout.strip().splitlines()[-1])
        res["one_thread"] = {"value": round(one["cmac"] / one["full_sample_s"] / 1e12, 7), "unit": "TCMAC/s",
                             "cores": 1,
                             "sample": f"the same subband on one thread: channeliser + requant on the first {S_1} "
                                       f"spectra ({one['ppf_requant_s']:.1f} s), correlator on 2 of 64 channels of "
                                       f"3051 spectra ({one['corr_s']:.1f} s), scaled to the full subband",
                             "speedup_of_all_threads": round(one["full_sample_s"] / main["total_s"], 2)}
    else:
        res["one_thread"] = {"error": (r.stderr or "sample is not the whole subband")[-300:]}
    # the whole 48-antenna configuration, float64 chain
    cfg = W.SMALL
    xs = W.make_voltages(cfg).numpy()[0]
    taps = W.prototype_taps()
    t0 = time.perf_counter()
    y = oracle.ppf_subband(xs, taps, 64, 16, cfg.n_spectra)
    t1 = time.perf_counter()
    for ch in range(64):
        oracle.xcorr(y[ch])
    t2 = time.perf_counter()
    n = cfg.n_inputs
    cm1 = 64.0 * n * (n + 1) // 2 * cfg.n_spectra
    res["small_whole"] = {"workload": cfg.name, "seconds": round(t2 - t0, 2), "ppf_s": round(t1 - t0, 2),
                          "correlator_s": round(t2 - t1, 2), "tcmacs": round(cm1 / (t2 - t0) / 1e12, 6),
                          "cmac": cm1}
    # the whole calibration configuration: loss and gradient at two gain sets
    Vc, Mc, gc = W.make_calibration(Na=576, P=64, seed=5)
    g1 = np.zeros_like(gc)
    g1[..., 0] = 1.0
    t0 = time.perf_counter()
    oracle.cal_loss_grad(Vc, Mc, gc)
    oracle.cal_loss_grad(Vc, Mc, g1)
    t1 = time.perf_counter()
    res["calibration_whole"] = {"workload": "576 antennas x 64 channels, XX and YY, true and unit gains",
                                "seconds": round(t1 - t0, 3), "seconds_per_evaluation": round((t1 - t0) / 2, 3)}
    return res


def chain_error(x0, vis_by_dtype, ants=PARITY_ANTENNAS):
    """Error of the GPU fp32 and fp16 chains of the timed run against the
    oracle's float64 chain on the same int16 samples (subband 0, the
    baselines among `ants`, all 64 channels): |V - V_ref| / sqrt(V_ii V_jj),
    max and RMS (the fp32 bar is 1e-5, the fp16 bar 2e-3)."""
    import numpy as np

    import oracle
    import workloads as W

    S = W.A12.n_spectra
    inputs = [2 * a + p for a in ants for p in range(2)]
    t0 = time.perf_counter()
    y = oracle.ppf_subband(x0, W.prototype_taps(), 64, 16, S, inputs=inputs)      # [P][S][R]
    pos = {i: k for k, i in enumerate(inputs)}
    pairs = np.array([(pos[2 * a + p], pos[2 * b + q]) for ia, a in enumerate(ants) for b in ants[: ia + 1]
                      for p in range(2) for q in range(2)])
    res = {"sample": f"subband 0 of the timed AARTFAAC-12 input, {len(ants)} antennas "
                     f"({len(pairs) // 4} baselines x 4 products), 64 channels, {S} spectra"}
    errs = {k: [] for k in vis_by_dtype}
    for ch in range(64):
        ref = oracle.xcorr_pairs(y[ch], pairs)
        pw = oracle.xcorr_pairs(y[ch], np.array([[k, k] for k in range(len(inputs))])).real
        den = np.sqrt(pw[pairs[:, 0]] * pw[pairs[:, 1]])
        for k, v in vis_by_dtype.items():
            errs[k].append(np.abs(v[ch].reshape(-1) - ref) / den)
    for k, e in errs.items():
        e = np.concatenate(e)
        res[k] = {"max": float(f"{e.max():.3e}"), "rms": float(f"{np.sqrt(np.mean(e * e)):.3e}"),
                  "bar": 1e-5 if k == "f32" else 2e-3}
    res["oracle_seconds"] = round(time.perf_counter() - t0, 2)
    return res


if __name__ == "__main__":
    if len(sys.argv) == 4 and sys.argv[1] == "--oracle-one-thread":
        _one_thread_child(int(sys.argv[2]), int(sys.argv[3]))
    else:
        main()
