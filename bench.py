#!/usr/bin/env python3
"""Encode/decode throughput of the DLIC hot path on one MI355X.

One step = encode the image (density kernel, rANS kernel, pack kernel),
fetch the stream length, decode it (wavefront kernel).  The input image is
resident in HBM before the timed region.  Prints one JSON line.

Workload (default): a 2048x1536 synthetic greyscale image (seed 1), network
12-64-64-15 FP32 (Glorot, seed 3), 64 groups x 4 interleaved rANS lanes (256
lanes), each group coding 2 row strips of 12 rows spread over the image.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_FP32_MFMA = 157.3e12
MI355X_BF16_MFMA = 2.5e15  # dense

# The paper's own timings, printed beside ours as context only: other hardware,
# other (trained, larger) networks, a softmax head and other images.
_MRI_PX = 256 * 256 * 35
_MRI_COMPLETE_S = [0.3374, 0.3946, 0.5997, 1.4250, 7.1203]
PAPER_CONTEXT = {
    "note": "context only, not a target: other hardware, networks, output head and data",
    "image_coding": {
        "hardware": "Ryzen 5 2600 CPU + GTX 1070 Ti GPU",
        "encode_s_per_image": "< 1 (smallest net, about 1e5 parameters; mean of 10 runs)",
        "decode_vs_encode": "within 4%",
        "source": "Section III-B, Fig. 3 (image and network sizes only in the figure)",
    },
    "mri_estimated": {
        "scan": "256x256x35, 12-bit",
        "params": [3.5e5, 1.35e6, 5.33e6, 1.75e7, 9.2e7],
        "first_frame_s": [0.2799, 0.3273, 0.4975, 1.1821, 5.9286],
        "complete_s": _MRI_COMPLETE_S,
        "complete_mpix_s": [round(_MRI_PX / t / 1e6, 3) for t in _MRI_COMPLETE_S],
        "hardware": "not named for these estimates",
        "source": "Section IV-D, Table III",
    },
}
MI355X_CUS = 256


def mlp_flops_per_px(h1, h2):
    return 2 * (12 * h1 + h1 * h2 + h2 * 15)


def schedule_bound_px(h, w, G, S=1):
    """Sum over wavefront steps of the largest per-group active pixel count (a group's
    S strips counted together)."""
    rows = [(b * h) // (G * S) for b in range(G * S + 1)]
    T = w + 3 * h - 3
    t = np.arange(T)
    worst = np.zeros(T, dtype=np.int64)
    for g in range(G):
        act = np.zeros(T, dtype=np.int64)
        for b in range(g, G * S, G):
            r0, r1 = rows[b], rows[b + 1]
            ylo = np.maximum(r0, np.floor_divide(t - w, 3) + 1)
            yhi = np.minimum(r1 - 1, np.floor_divide(t, 3))
            act += np.maximum(0, yhi - ylo + 1)
        worst = np.maximum(worst, act)
    return int(worst.sum())


def step_chain_cycles(probe, hidden):
    """Shader cycles of the dependent operations one wavefront step needs for one
    row, each at its measured latency (probe: dlic_latency_probe's cycles per
    link), with every independent operation assumed in parallel and no hand-off
    between waves.  Returns (density part, coder part, breakdown).

    density: the left neighbour, decoded in the step before, is read back from
    LDS (store then load) and scaled (3 ops); layer 1's chain ends with the up-right
    neighbour and the two left ones (3 FMAs) and a ReLU; layer 1's outputs reach
    layer 2's lanes through LDS; layer 2 is one FMA chain over all H inputs in the
    format's order, then ReLU and LDS again; layer 3 is a chain over one K quarter
    (H / 4 inputs; the whole H at 32 wide) and three adds joining the quarters;
    the head takes a maximum over 5 logits (4 ops), one exponential, a 5-term sum
    (4 adds), a reciprocal (2 ops) and a product; its parameters reach the
    table lanes through LDS; a bucket boundary is the table rule at one level:
    u = beta A + B, clamp, integer and fraction (6 ops), one table load from LDS,
    the interpolation (2), the 5-component sum (4 deep) and F (3).
    coder: the slot against the boundaries (1) and a 16-lane reduction, the
    table rule at the level inside the bucket as above, a second comparison and
    reduction, the rANS update, and the renormalisation (ballot, popcount,
    readlane and a select)."""
    fma, lsl, ld = probe["fma_f32"], probe["lds_store_load"], probe["lds_load"]
    layer3 = hidden // 4 + 3 if hidden >= 64 else hidden
    table = 6 * fma + ld + 2 * fma + 4 * fma + 3 * fma
    parts = {
        "window": lsl + 3 * fma,
        "layer1_tail": 3 * fma + fma,
        "layer2": lsl + hidden * fma + fma,
        "layer3": lsl + layer3 * fma,
        "head": 4 * fma + probe["expf"] + 4 * fma + 2 * fma + fma,
        "boundaries": lsl + table,
    }
    coder = {
        "bucket": fma + probe["dpp_reduce16"],
        "level": table,
        "symbol": fma + probe["dpp_reduce16"],
        "update": probe["rans_update"] + probe["ballot_popcount"] + probe["readlane"] + fma,
    }
    return sum(parts.values()), sum(coder.values()), {**parts, **{"coder_" + k: v for k, v in coder.items()}}


def decode_latency_bound_ms(probe, H, W, G, L, hidden, S=1):
    """Lower bound on the decode time from dependent latencies: every one of the
    T = W + 3H - 3 wavefront steps waits for the step before it (left and up-right
    neighbours), a lane decodes its J = ceil(rows per strip / L) rows of a step one
    after another (its state carries from row to row), and each of the G*S - 1
    strip boundaries on the critical path passes a pixel between workgroups
    through device memory instead of LDS."""
    dens, coder, parts = step_chain_cycles(probe, hidden)
    T = W + 3 * H - 3
    J = -(-(-(-H // (G * S))) // L)
    per_step = max(J * coder, dens + coder)
    cross = (G * S - 1) * max(0.0, probe["global_flag_handoff"] - probe["lds_store_load"])
    cycles = T * per_step + cross
    return cycles / (probe["shader_clock_mhz"] * 1e3), {
        "steps": T, "rows_per_lane_per_step": J, "density_chain_cycles": dens,
        "coder_chain_cycles": coder, "per_step_cycles": per_step,
        "group_crossing_cycles": cross, "chain_cycles": parts}


def host_info():
    """CPU model, core counts and the BLAS the oracle's matrix products use."""
    from threadpoolctl import threadpool_info
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads"),
             "version": d.get("version")} for d in threadpool_info() if d.get("user_api") == "blas"]
    return {"cpu": model, "os_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "blas": blas}


def cpu_baseline(img, weights, groups, lanes, strips=1, target_s=15.0):
    """Time the oracle's encode and decode on a crop of the image: the encoder's
    network as BLAS matrix products on every core this process may use, its rANS
    walk in one Python thread, the per-pixel decoder in one thread (BLAS too)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle
    n_threads = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=n_threads, user_api="blas"):
        used = max([d.get("num_threads") or 1 for d in threadpool_info()
                    if d.get("user_api") == "blas"] or [1])
        # size the crop so the run takes roughly target_s
        probe = np.ascontiguousarray(img[:16, :128])
        t0 = time.perf_counter()
        b = oracle.encode_image(probe, weights, oracle.OracleCoder(1, lanes))
        with threadpool_limits(limits=1, user_api="blas"):
            oracle.decode_image(b, weights)
        per_px = (time.perf_counter() - t0) / probe.size
        n_px = int(min(img.size, max(4096, target_s / max(per_px, 1e-9))))
        cw = min(img.shape[1], 512)
        ch = max(2, min(img.shape[0], n_px // cw))
        crop = np.ascontiguousarray(img[:ch, :cw])
        g = max(1, min(groups, ch // 2))
        coder = oracle.OracleCoder(g, lanes, max(1, min(strips, ch // (2 * g))))
        t0 = time.perf_counter()
        bits = oracle.encode_image(crop, weights, coder)
        t1 = time.perf_counter()
    # the decoder's products have one row each: more BLAS threads only add overhead
    with threadpool_limits(limits=1, user_api="blas"):
        t1 = time.perf_counter()
        dec = oracle.decode_image(bits, weights)
        t2 = time.perf_counter()
    assert np.array_equal(dec, crop)
    te, td = t1 - t0, t2 - t1
    return {"value": crop.size / (te + td) / 1e6, "unit": "MPix/s", "cores": used,
            "kind": "oracle",
            "encode_mpix_s": crop.size / te / 1e6, "decode_mpix_s": crop.size / td / 1e6,
            "sample": f"oracle encode then decode of the top-left {ch}x{cw} crop of the same "
                      f"image ({coder.groups}x{lanes} lanes, {coder.strips} strips per group): "
                      f"network products through BLAS on "
                      f"{used} threads in encode, rANS and the per-pixel decode in one thread; encode "
                      f"{te:.1f} s, decode {td:.1f} s"}


def kernel_sources_sha256() -> str:
    """Digest of the HIP sources; counter readings are valid only for the code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2207_05152_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of a kernel from the committed counter summary
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE per dispatch, each scaled
    by what the same counter read for a plain copy of known size), or None when
    the kernels changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_sources_sha256() or kernel not in t.get("kernels", {}):
        return None
    return float(t["kernels"][kernel]["bytes_per_launch"])


def precision_sweep(dl, torch, img, H, W, coder, hidden=128, reps=3):
    """Encode + decode of the same image with the 12-128-128-15 net stored as
    FP32, BF16 and FP8 e4m3: kernel-timed MPix/s, bpp and the bpp change
    against FP32 (outside the timed region of the main step)."""
    import synth
    weights = synth.xavier_mlp((12, hidden, hidden, 15), 3)
    n_px = H * W
    cap = dl.dlic_encode_bound(H, W, coder)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    olen = torch.zeros(1, dtype=torch.int64, device="cuda")
    ews = torch.empty(dl.dlic_encode_workspace(H, W, coder), dtype=torch.uint8, device="cuda")
    dws = torch.empty(dl.dlic_decode_workspace(H, W, coder), dtype=torch.uint8, device="cuda")
    dec = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    # W8A8 activation multipliers from calibration images disjoint from the workload
    cal = [torch.from_numpy(synth.synth_image(256, 256, seed)).cuda() for seed in range(1000, 1008)]
    dl.dlic_set_timing(True)
    for dtype in ("fp32", "bf16", "fp8", "fp8a8"):
        model = dl.Model(weights, "cuda:0", dtype=dtype, calibration=cal)
        dl.dlic_set_timing(True)
        kt = {}
        for r in range(reps + 1):
            dl.dlic_encode(model.c, coder, img, H, W, out, cap, olen, ews, ews.numel(), stream)
            ke = dict(dl.dlic_kernel_times())
            n = int(olen.item())
            dl.dlic_decode(model.c, coder, out, n, dec, H, W, st, dws, dws.numel(), stream)
            kd = dict(dl.dlic_kernel_times())
            if r:
                for k, v in list(ke.items()) + list(kd.items()):
                    kt.setdefault(k, []).append(v)
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and torch.equal(dec, img), f"{dtype} round trip failed"
        avg = {k: float(np.mean(v)) for k, v in kt.items()}
        enc = avg["density_kernel"] + avg["rans_encode_kernel"] + avg["pack_kernel"]
        dcd = avg["wavefront_decode_kernel"] + avg.get("fill_u32_kernel", 0.0)
        res[dtype] = {"encode_mpix_s": n_px / enc / 1e3, "decode_mpix_s": n_px / dcd / 1e3,
                      "density_ms": avg["density_kernel"], "decode_ms": dcd,
                      "bpp_total": 8.0 * n / n_px}
    dl.dlic_set_timing(False)
    for dtype in ("bf16", "fp8", "fp8a8"):
        res[dtype]["bpp_delta_vs_fp32"] = res[dtype]["bpp_total"] - res["fp32"]["bpp_total"]
    res["bf16_gate_0.01bpp"] = abs(res["bf16"]["bpp_delta_vs_fp32"]) <= 0.01
    # BF16 over FP32 on the same GPU, image and layout (kernel times)
    res["bf16_speedup_vs_fp32"] = {
        d: res["bf16"][f"{d}_mpix_s"] / res["fp32"][f"{d}_mpix_s"] for d in ("encode", "decode")}
    res["workload"] = (f"{W}x{H} image (seed 1), MLP 12-{hidden}-{hidden}-15 (Glorot seed 3) "
                       f"stored as FP32 / BF16 / FP8 e4m3 weights with per-layer scales (BF16 "
                       f"activations) / FP8 weights and activations (activation multipliers "
                       f"calibrated on 8 images, seeds 1000-1007), "
                       f"{coder.groups}x{coder.lanes_per_group} lanes, "
                       f"{max(1, coder.strips)} row strips per group")
    return res


def layout_sweep(dl, torch, img, H, W, model, probe, hidden,
                 layouts=((64, 4, 1), (64, 4, 3), (64, 4, 4), (128, 2, 1), (128, 2, 2),
                          (8, 32, 1), (16, 16, 1), (32, 8, 1), (256, 1, 1), (128, 4, 1),
                          (128, 4, 2), (192, 4, 1), (384, 4, 1), (48, 32, 1)), reps=3):
    """The main step's image and net coded with other coder layouts (G groups x L
    lanes x S row strips per group).  Those up to 256 x 1 have the main step's 256
    lanes; the decoder gives a pixel 16 coder lanes when L <= 4.  Strips spread
    over the image, and more lanes, cut the sequential sub-rounds per wavefront
    step, ceil(rows per strip / L); more lanes cost 4 flushed bytes per lane;
    384 x 4 and 48 x 32 give every row its own lane (one sub-round per step)."""
    out = []
    dl.dlic_set_timing(True)
    for G, L, S in layouts:
        coder = dl.dlic_coder(G, L, S)
        bits = dl.encode(img, model, coder)
        dec = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = torch.empty(dl.dlic_decode_workspace(H, W, coder), dtype=torch.uint8, device="cuda")
        ms = []
        for r in range(reps + 1):
            dl.dlic_decode(model.c, coder, bits, bits.numel(), dec, H, W, st, ws, ws.numel())
            if r:
                ms.append(dict(dl.dlic_kernel_times())["wavefront_decode_kernel"])
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and torch.equal(dec, img), f"layout {G}x{L}x{S} round trip"
        rows = -(-H // (G * S))
        bound_ms, _ = decode_latency_bound_ms(probe, H, W, G, L, hidden, S)
        out.append({"groups": G, "lanes": L, "strips": S, "sub_rounds_per_step": -(-rows // L),
                    "decode_ms": float(np.mean(ms)), "decode_mpix_s": H * W / np.mean(ms) / 1e3,
                    "latency_bound_ms": bound_ms, "frac_latency": bound_ms / float(np.mean(ms)),
                    "bpp_total": 8.0 * bits.numel() / (H * W)})
    dl.dlic_set_timing(False)
    return out


def _synth_job(args):
    import synth
    h, w, seed = args
    return synth.synth_image(h, w, seed)


def batch_sweep(dl, torch, reps=3, tune_budget_s=60.0):
    """The 64-image batch (seeds 100..163, sizes drawn from 256x256 .. 2048x1536)
    with the 12-64-64-15 net in BF16: autotuned knobs, one captured graph per
    direction, aggregate MPix/s, per-image latency percentiles, bpp."""
    from concurrent.futures import ProcessPoolExecutor

    import synth
    from paper_2207_05152_amd import autotune
    seeds = list(range(100, 164))
    sizes = synth.batch_sizes(seeds)
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        images = list(ex.map(_synth_job, [(h, w, sd) for (h, w), sd in zip(sizes, seeds)]))
    model = dl.Model(synth.xavier_mlp((12, 64, 64, 15), 3), "cuda:0", dtype="bf16")
    n_px = sum(h * w for h, w in sizes)
    tuned = autotune.tune(model, sizes, images, budget_s=tune_budget_s)

    def run(knobs):
        b = dl.Batch(model, sizes, coders=autotune.coders_for(sizes, knobs["rows_per_group"],
                                                                knobs["lanes"]),
                     density_grid=knobs["density_grid"],
                     search_lanes=knobs.get("search_lanes", 0),
                     decode_grid=knobs.get("decode_grid", 0))
        b.load(images)
        b.capture()
        s = torch.cuda.current_stream()
        b.replay(False, s)
        b.replay(True, s)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        enc, dec, lat_e, lat_d = [], [], [], []
        for _ in range(reps):
            ev[0].record(s)
            b.replay(False, s)
            ev[1].record(s)
            b.replay(True, s)
            ev[2].record(s)
            torch.cuda.synchronize()
            enc.append(ev[0].elapsed_time(ev[1]))
            dec.append(ev[1].elapsed_time(ev[2]))
            lat_e.append(b.latencies_s(False))
            lat_d.append(b.latencies_s(True))
        assert bool((b.status == 0).all().item()), "batch decode status"
        assert torch.equal(b.decoded, b.pixels), "batch round trip is not lossless"
        nbytes = int(b.lens.sum().item())
        le, ld = np.concatenate(lat_e) * 1e3, np.concatenate(lat_d) * 1e3
        out = {"encode_ms": float(np.mean(enc)), "decode_ms": float(np.mean(dec)),
               "encode_mpix_s": n_px / np.mean(enc) / 1e3, "decode_mpix_s": n_px / np.mean(dec) / 1e3,
               "encode_latency_ms_p50_p99": [float(np.percentile(le, 50)), float(np.percentile(le, 99))],
               "decode_latency_ms_p50_p99": [float(np.percentile(ld, 50)), float(np.percentile(ld, 99))],
               "bpp_total": 8.0 * nbytes / n_px, "groups": int(sum(c[0] for c in b.coders)),
               "knobs": knobs}
        b.close()
        return out

    res = {"workload": f"64 synthetic images (seeds 100-163, sizes from 256x256 to 2048x1536, "
                       f"{n_px / 1e6:.1f} Mpx), MLP 12-64-64-15 BF16 (Glorot seed 3); one captured "
                       f"graph per direction",
           "tuned": run(tuned["knobs"]), "default": run(dict(autotune.DEFAULT)),
           "autotune": {"key": tuned["key"], "cached": tuned["cached"],
                        "trials": len(tuned["trials"])}}
    return res


def deep_flops_per_px(hidden, k_in=12, n_out=256):
    """FLOP per pixel of the six-layer k_in -> H x 5 -> n_out network (2 per MAC)."""
    return 2 * (k_in * hidden + 4 * hidden * hidden + hidden * n_out)


def deep_sweep(dl, torch, img, H, W, hidden=128, layout=(48, 32), reps=2):
    """The paper's own network and head (six dense layers, softmax over 256 levels), BF16
    weights, on the same image: encode and decode kernel times, MPix/s, bpp and the
    encoder density kernel's MFMA rate (outside the timed region of the main step)."""
    import synth
    m = dl.DeepModel(synth.xavier_deep(hidden, 3), "cuda:0")
    coder = dl.dlic_coder(*layout)
    dl.dlic_set_timing(True)
    kt = {}
    for r in range(reps + 1):
        bits = dl.deep_encode(img, m, coder)
        ke = dict(dl.dlic_kernel_times())
        dec, st = dl.deep_decode(bits, m, check=False)
        kd = dict(dl.dlic_kernel_times())
        if r:
            for k, v in list(ke.items()) + list(kd.items()):
                kt.setdefault(k, []).append(v)
    torch.cuda.synchronize()
    dl.dlic_set_timing(False)
    assert st == 0 and torch.equal(dec, img), "softmax-network round trip"
    avg = {k: float(np.mean(v)) for k, v in kt.items()}
    enc = avg["deep_density_kernel"] + avg["rans_encode_kernel"] + avg["pack_kernel"]
    dcd = avg["deep_decode_kernel"]
    n_px = H * W
    flop = n_px * deep_flops_per_px(hidden)
    return {"workload": f"{W}x{H} image (seed 1), six dense layers 12-{hidden}x5-256 with a "
                        f"softmax over 256 levels, BF16 weights (Glorot seed 3), "
                        f"{layout[0]}x{layout[1]} lanes",
            "params": int(sum(W_.size + b.size for W_, b in synth.xavier_deep(hidden, 3))),
            "kernel_ms": avg, "encode_mpix_s": n_px / enc / 1e3, "decode_mpix_s": n_px / dcd / 1e3,
            "bpp_total": 8.0 * bits.numel() / n_px,
            "density_tflops": flop / (avg["deep_density_kernel"] * 1e-3) / 1e12,
            "density_frac_bf16_mfma": flop / (avg["deep_density_kernel"] * 1e-3) / MI355X_BF16_MFMA,
            "decode_us_per_step": dcd * 1e3 / (W + 3 * H - 3)}


def volume_sweep(dl, torch, hidden=128, Z=35, size=256, layout=(8, 8), shifts=(0, 1, 2), reps=2):
    """Volumes (3-D window and 3-D wavefront) on a 256x256x35 phantom scan, the six-layer
    network with 21 inputs: encode and decode kernel times per window shift, MPix/s, bpp,
    the step at which the first slice is complete; the same scan with a 12-input
    network, once with all slices in one 3-D wavefront and once slice by slice through the
    image decoder; and the 12-bit scan with 4096 output levels (outside the timed region of
    the main step)."""
    import synth
    vol = torch.from_numpy(synth.mri_volume(2024, depth=Z, size=size)).cuda()
    vol12 = torch.from_numpy(synth.mri_volume(2024, depth=Z, size=size, bits=12).astype(np.int16)).cuda()
    n_px = vol.numel()
    coder = dl.dlic_coder(*layout)
    T2 = size + 3 * (size - 1)

    def run(m, ws, vol=vol):
        dl.dlic_set_timing(True)
        kt = {}
        for r in range(reps + 1):
            bits = dl.volume_encode(vol, m, coder, ws)
            ke = dict(dl.dlic_kernel_times())
            dec, st = dl.volume_decode(bits, m, check=False)
            kd = dict(dl.dlic_kernel_times())
            if r:
                for k, v in list(ke.items()) + list(kd.items()):
                    kt.setdefault(k, []).append(v)
        torch.cuda.synchronize()
        dl.dlic_set_timing(False)
        assert st == 0 and torch.equal(dec, vol), "volume round trip"
        avg = {k: float(np.mean(v)) for k, v in kt.items()}
        d12 = m.depth == 12
        stamps = {}
        if not d12:
            # device real-time stamps of the last decode: start, each slice done
            s_ = dl.dlic_deep_slice_stamps(Z + 1).astype(np.int64)
            hz = dl.dlic_wallclock_hz()
            first = (s_[1] - s_[0]) / hz * 1e3
            complete = (s_[1:].max() - s_[0]) / hz * 1e3
            stamps = {"first_slice_ms": first, "complete_ms": complete,
                      "first_over_complete": first / complete}
        dens = avg["deep12_density" if d12 else "deep_density_kernel"]
        enc = dens + avg["rans_encode_kernel"] + avg["pack_kernel"]
        dcd = avg["deep12_decode_kernel" if d12 else "deep_decode_kernel"]
        lag = max(0, 3 * ws - 1) if m.k_in == 21 else 0
        T = T2 + lag * (Z - 1)
        flop = n_px * deep_flops_per_px(hidden, m.k_in, 1 << m.depth)
        return {"kernel_ms": avg, "encode_mpix_s": n_px / enc / 1e3,
                "decode_mpix_s": n_px / dcd / 1e3, "decode_ms": dcd,
                "bpp_total": 8.0 * bits.numel() / n_px, "lag": lag, "steps": T,
                "first_slice_steps": T2, "decode_grid": dl.dlic_deep_decode_grid(),
                "decode_us_per_step": dcd * 1e3 / T, **stamps,
                "density_tflops": flop / (dens * 1e-3) / 1e12,
                "density_frac_bf16_mfma": flop / (dens * 1e-3) / MI355X_BF16_MFMA}

    m3 = dl.DeepModel(synth.xavier_deep(hidden, 3, k_in=21), "cuda:0")
    out = {"workload": f"{size}x{size}x{Z} phantom scan (seed 2024), six dense layers "
                       f"21-{hidden}x5-256 with a softmax over 256 levels, BF16 weights (Glorot "
                       f"seed 3), {layout[0]} groups x {layout[1]} lanes per slice",
           "params": int(sum(W_.size + b.size for W_, b in synth.xavier_deep(hidden, 3, k_in=21))),
           "window_shift": {}}
    for ws in shifts:
        out["window_shift"][str(ws)] = run(m3, ws)
    m2 = dl.DeepModel(synth.xavier_deep(hidden, 3, k_in=12), "cuda:0")
    out["slices_in_one_wavefront_12_inputs"] = run(m2, 0)
    # the same slices one image at a time through the image decoder
    bits = [dl.deep_encode(vol[z], m2, coder) for z in range(Z)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for z in range(Z):
        dec, st = dl.deep_decode(bits[z], m2, check=False)
    torch.cuda.synchronize()
    out["slice_by_slice_12_inputs_decode_ms"] = (time.perf_counter() - t0) * 1e3
    m12 = dl.DeepModel(synth.xavier_deep(hidden, 3, k_in=21, n_out=4096), "cuda:0")
    out["bits12_window_shift_1"] = run(m12, 1, vol12)
    out["bits12_params"] = int(sum(W_.size + b.size for W_, b in
                                   synth.xavier_deep(hidden, 3, k_in=21, n_out=4096)))
    return out


def _phantom_job(seed):
    import synth
    return synth.mri_phantom(seed, 256)


def training_sweep(dl, torch, steps=20, n=1 << 20):
    """Retraining steps on MRI-like slices: 2^20 sampled windows per step from a
    256-slice 256x256 phantom stack, 12-64-64-15 FP32, hand-written loss+gradient
    kernel then Adam; steps/s and MFMA rate (forward + backward ~ 3x forward FLOP)."""
    from concurrent.futures import ProcessPoolExecutor

    import synth
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        stack = np.stack(list(ex.map(_phantom_job, range(2000, 2256))))
    slices = torch.from_numpy(stack).cuda()
    model = dl.TrainModel(synth.xavier_mlp((12, 64, 64, 15), 3), "cuda")
    idx = [torch.from_numpy(synth.train_indices(k, n, 256, 256, 256)).cuda() for k in range(steps)]
    npar = model.flat.numel()
    m = torch.zeros_like(model.flat)
    v = torch.zeros_like(model.flat)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(model.flat)
    wsb = dl.dlic_nll_workspace(n, model.c)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    losses = []

    def one(k):
        dl.dlic_nll_fwd_bwd(model.c, slices, 256, 256, 256, idx[k], n, loss, grad, ws, wsb)
        dl.dlic_adam_step(npar, model.flat, grad, m, v, k + 1)

    one(0)
    losses.append(float(loss.item()))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps):
        one(k)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / (steps - 1)
    losses.append(float(loss.item()))
    flop = 3 * n * mlp_flops_per_px(64, 64)
    return {"workload": f"{n} windows per step from 256 phantom slices of 256x256, MLP 12-64-64-15 "
                        f"FP32 (Glorot seed 3), loss + gradient kernel then Adam",
            "ms_per_step": dt * 1e3, "steps_per_s": 1.0 / dt, "samples_per_s": n / dt,
            "tflops_approx": flop / dt / 1e12, "frac_fp32_mfma": flop / dt / MI355X_FP32_MFMA,
            "loss_bits_first_last": losses}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--height", type=int, default=1536)
    ap.add_argument("--width", type=int, default=2048)
    ap.add_argument("--hidden", type=int, default=64)
    ap.add_argument("--groups", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--strips", type=int, default=2, help="row strips per group")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed steps, run one plain elementwise copy of MIB MiB "
                         "(FP32 negation) so that counter runs can scale FETCH_SIZE/WRITE_SIZE")
    ap.add_argument("--no-decode-profile", action="store_true",
                    help="skip the extra decode with the in-kernel cycle counters (so that a "
                         "profiler's kernel averages cover the timed launches only)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision, batch and training sweeps after the main step")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the DLIC hot path here runs on a single MI355X "
              "(no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2207_05152_amd as dl
    import synth

    torch.cuda.set_device(0)
    dl.dlic_init(0)
    H, W, Hd = args.height, args.width, args.hidden
    img_np = synth.synth_image(H, W, 1)
    weights = synth.xavier_mlp((12, Hd, Hd, 15), 3)
    model = dl.Model(weights, "cuda:0")
    coder = dl.dlic_coder(args.groups, args.lanes, args.strips)
    img = torch.from_numpy(img_np).cuda()
    n_px = H * W

    cap = dl.dlic_encode_bound(H, W, coder)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    olen = torch.zeros(1, dtype=torch.int64, device="cuda")
    ews = torch.empty(dl.dlic_encode_workspace(H, W, coder), dtype=torch.uint8, device="cuda")
    dws = torch.empty(dl.dlic_decode_workspace(H, W, coder), dtype=torch.uint8, device="cuda")
    dec = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    kt = {}

    def step(record):
        dl.dlic_encode(model.c, coder, img, H, W, out, cap, olen, ews, ews.numel(), stream)
        if record:
            for name, ms in dl.dlic_kernel_times():
                kt.setdefault(name, []).append(ms)
        n = int(olen.item())
        dl.dlic_decode(model.c, coder, out, n, dec, H, W, st, dws, dws.numel(), stream)
        if record:
            for name, ms in dl.dlic_kernel_times():
                kt.setdefault(name, []).append(ms)
        return n

    if args.calibrate_copy > 0:
        n_el = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    dl.dlic_set_timing(True)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        n_bytes = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dl.dlic_set_timing(False)

    # one more decode with the in-kernel cycle counters on (outside the timed region)
    prof = torch.zeros(16 * args.groups, dtype=torch.int64, device="cuda")
    if not args.no_decode_profile:
        dl.dlic_set_decode_profile(prof)
        dl.dlic_decode(model.c, coder, out, n_bytes, dec, H, W, st, dws, dws.numel(), stream)
        torch.cuda.synchronize()
        dl.dlic_set_decode_profile(None)
    pc = prof.view(args.groups, 16).cpu().numpy().astype(np.float64)
    busy = pc[:, 0] + pc[:, 1]
    tiles = max(pc[:, 7].sum(), 1)
    decode_profile = {
        "coder_wait_frac": float(pc[:, 0].sum() / max(busy.sum(), 1)),
        "worker_wait_frac": float(pc[:, 2].sum() / max((pc[:, 2] + pc[:, 3]).sum(), 1)),
        "coder_cycles_per_group": [int(v) for v in busy],
        "worker_cycles_per_tile": {"gather_net": float(pc[:, 4].sum() / tiles),
                                   "head": float(pc[:, 5].sum() / tiles),
                                   "buckets_publish": float(pc[:, 6].sum() / tiles),
                                   "tiles": int(tiles)},
        "shader_clock_mhz": float(pc[:, 13].sum() / max(pc[:, 14].sum(), 1) * 100.0),
        "coder_loop_cycles_per_sub_round": float(pc[:, 13].sum() / max(pc[:, 10].sum(), 1)),
        "coder_cycles_per_sub_round": {"busy": float(pc[:, 1].sum() / max(pc[:, 10].sum(), 1)),
                                       "to_search": float(pc[:, 8].sum() / max(pc[:, 10].sum(), 1)),
                                       "search": float(pc[:, 9].sum() / max(pc[:, 10].sum(), 1))},
    }

    assert int(st.item()) == 0, f"decode status {int(st.item())}"
    assert torch.equal(dec, img), "round trip is not lossless"

    avg = {k: float(np.mean(v)) for k, v in kt.items()}
    enc_ms = avg.get("density_kernel", 0) + avg.get("rans_encode_kernel", 0) + avg.get("pack_kernel", 0)
    dec_ms = avg.get("wavefront_decode_kernel", 0) + avg.get("fill_u32_kernel", 0)
    ms_step = elapsed / args.steps * 1e3
    flops = n_px * mlp_flops_per_px(Hd, Hd)
    dom = max(avg, key=avg.get)
    dom_flops = flops if dom in ("wavefront_decode_kernel", "density_kernel") else 0
    achieved = dom_flops / (avg[dom] * 1e-3) if dom_flops else 0.0
    crit_px = schedule_bound_px(H, W, args.groups, args.strips)
    sched_ms = crit_px * mlp_flops_per_px(Hd, Hd) / (MI355X_FP32_MFMA / MI355X_CUS) * 1e3
    steps_T = W + 3 * (H - 1)
    J = -(-(-(-H // (args.groups * args.strips))) // args.lanes)
    crit_sub = steps_T * J

    probe = dl.dlic_latency_probe()
    lat_ms, lat_detail = decode_latency_bound_ms(probe, H, W, args.groups, args.lanes, Hd,
                                                 args.strips)
    dec_kernel_ms = avg.get("wavefront_decode_kernel")

    res = {
        "metric": "encode/decode MPix/s on 1 MI355X + bpp; BF16 vs FP32 at \u22640.01 bpp \u0394",
        "value": n_px / (ms_step * 1e-3) / 1e6,
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{W}x{H} synthetic greyscale image (seed 1), MLP 12-{Hd}-{Hd}-15 FP32 "
                        f"(Glorot seed 3), {args.groups} groups x {args.lanes} rANS lanes, "
                        f"{args.strips} row strips per group; one step = encode + decode",
            "image": [H, W], "hidden": Hd, "groups": args.groups, "lanes_per_group": args.lanes,
            "strips_per_group": args.strips,
        },
        "encode_mpix_s": n_px / (enc_ms * 1e-3) / 1e6 if enc_ms else None,
        "decode_mpix_s": n_px / (dec_ms * 1e-3) / 1e6 if dec_ms else None,
        "bpp_total": 8.0 * n_bytes / n_px,
        "bpp_payload": 8.0 * (n_bytes - 36 - 4 * args.groups) / n_px,
        "kernel_ms": avg,
        "roofline": {
            "kernel": dom,
            "bound": "mfma",
            "achieved": achieved / 1e12,
            "peak": MI355X_FP32_MFMA / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / MI355X_FP32_MFMA,
            "traffic": measured_traffic(dom),
            "latency_bound_ms": lat_ms,
            "frac_latency": (lat_ms / dec_kernel_ms) if dec_kernel_ms else None,
            "note": "bound/peak/frac: the chip's FP32 MFMA peak; the decode is latency-bound, "
                    "and frac_latency is the decode bound built from the measured latencies of "
                    "its dependent operations (latency_probe, decode_latency) over the measured "
                    "decode kernel time",
        },
        "decode_latency": lat_detail,
        "decode_span": {
            "wavefront_steps": steps_T,
            "sub_rounds_per_step": J,
            "critical_sub_rounds": crit_sub,
            "ns_per_sub_round": (avg["wavefront_decode_kernel"] * 1e6 / crit_sub
                                 if "wavefront_decode_kernel" in avg else None),
            "mfma_bound_ms": sched_ms,
            "note": "groups move in lock-step on the wavefront step and each step is J sequential "
                    "coder sub-rounds, so decode time is critical_sub_rounds x the coder's "
                    "sub-round latency; mfma_bound_ms is the density work on that path at one "
                    "CU's FP32 MFMA peak per group",
        },
        "decode_profile": decode_profile,
        "latency_probe": probe,
        "host": host_info(),
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_extras:
        res["layouts"] = layout_sweep(dl, torch, img, H, W, model, probe, Hd)
        res["precision"] = precision_sweep(dl, torch, img, H, W, coder)
        res["batch"] = batch_sweep(dl, torch)
        res["training"] = training_sweep(dl, torch)
        res["softmax_net"] = deep_sweep(dl, torch, img, H, W)
        res["volume"] = volume_sweep(dl, torch)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(img_np, weights, args.groups, args.lanes, args.strips)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
