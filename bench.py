"""Benchmark of the ratio-filter hot path on one MI355X.

Headline workload: batched uneven -- 8 data segments of 256 s at 4096 Hz
(2^20 samples each), f_low = 25 Hz, 64 references with m1, m2 ~ U[1, 3] Msun,
each with floor(exp U[ln 32, ln 512]) lattice neighbours (10,136 kernels in
all), coloured Gaussian noise plus one injection per segment (synthetic,
seeded).  The largest configuration that fits one GPU.

One step = the method's whole per-batch work: the reference matched filter of
every (segment, reference) (FP64 TaylorF2 spectrum + FP32 FFT), and the
split-FP16 reconstruction of every neighbour series of every segment in one
persistent launch with the fused peak / threshold read-out (|z| > 6), captured
in hipGraphs and replayed.  value = produced template-SNR samples per second,
(kernels + references) * n * segments / step time.  Kernel build is timed
separately (it is done once and stored).

Beside it (under "extra"): the single-reference realistic workload (512 s,
256 neighbours) with the plain FP32 path, direct FFT matched filtering of the
same templates, the factored and overlap-save forms, bank organisation, the
reduced batched launch against its call loop, the learned kernels, and the
next-generation-detector shape (2048 s, 4 x 1024 templates).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2511_12894_amd import rf, synth  # noqa: E402

METRIC = "reconstructed template-SNR samples/s vs direct FFT MF at ≤2e-4 err; %roofline"
PEAK_FP16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3          # FP32 matrix cores (v_mfma_f32_32x32x2_f32)
PEAK_FP32_VECTOR_TFLOPS = 78.6    # FP32 vector ALU without packed-FP32 instructions (the build disables them)
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(fn, steps, warmup, stream):
    """Run fn warmup + steps times; return (total ms of the timed steps, per-call ms list)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return wall, [a.elapsed_time(b) for a, b in evs]


def counter_summary(name):
    """The committed rocprofv3 counter summary profiles/<name>_counters.json, or
    None when any source the kernel is built from (the files listed there,
    headers included) changed since the counters were taken."""
    import hashlib
    try:
        d = json.load(open(os.path.join(ROOT, "profiles", f"{name}_counters.json")))
        for rel, digest in d["sources_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest() != digest:
                return None
        float(d["traffic_bytes_per_dispatch"])
    except (OSError, ValueError, KeyError, AttributeError, TypeError):
        return None
    return d


def counter_traffic(name):
    """Calibrated HBM bytes per launch of a kernel from its counter summary (None as above)."""
    d = counter_summary(name)
    return None if d is None else float(d["traffic_bytes_per_dispatch"])


def host_cpu():
    """(model name, usable cores) of the host this runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def _oracle_group(args):
    """Oracle work of one reference group on one segment: the reference's
    matched filter and the FFT-based reconstruction of the given neighbours
    (kernels built beforehand, untimed).  Returns the seconds it took."""
    from oracle import mf as omf
    from oracle import ratio as orat
    g, xf, psd, ref, kern = args
    t0 = time.perf_counter()
    zr, nr = omf.grid_snr_series(g, xf, psd, *ref)
    for m_lo, taps, scale in kern:
        orat.reconstruct(zr, m_lo, taps, nr * scale)
    return time.perf_counter() - t0


def cpu_baseline_batched(wb, n_groups_1=2, per_group=6, seed=77):
    """The FP64 oracle on the host on a seeded subset of the batched workload:
    reference groups of segment 0 (reference matched filter + FFT-based
    reconstruction of `per_group` seeded neighbours each, full 2^20-sample
    series).  Single core: n_groups_1 groups in this process; all cores: one
    group per usable core in a process pool.  Rates are extrapolated to the
    whole workload as template-samples per second (kernel builds untimed)."""
    import multiprocessing as mp
    from oracle import mf as omf
    from oracle import ratio as orat
    g = wb["grid"]
    psd = wb["psd"]
    xf = wb["segments"][0]
    model, cores = host_cpu()
    ncores = max(1, min(cores, 16))
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(wb["refs"]), size=max(n_groups_1, ncores), replace=ncores > len(wb["refs"]))
    tasks = []
    for r in pick:
        ref = wb["refs"][int(r)]
        grp = wb["groups"][int(r)]
        sel = rng.choice(len(grp), size=min(per_group, len(grp)), replace=False)
        kern = []
        for i in sel:
            nb = grp[int(i)]
            kb = orat.build_kernel(g, ref, nb)
            nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, psd, omf.template_spectrum(g.fs, g.n, *nb))
            kern.append((kb["m_lo"], kb["taps"], 1.0 / nk))
        tasks.append((g, xf, psd, ref, kern))
    t0 = time.perf_counter()
    for t in tasks[:n_groups_1]:
        _oracle_group(t)
    t1 = time.perf_counter() - t0
    tmpl1 = sum(1 + len(t[4]) for t in tasks[:n_groups_1])
    single = tmpl1 * g.n / t1
    with mp.get_context("fork").Pool(ncores) as pool:
        pool.map(_oracle_group, tasks[:1])                 # start the workers
        t0 = time.perf_counter()
        pool.map(_oracle_group, tasks[:ncores], chunksize=1)
        tn = time.perf_counter() - t0
    tmpln = sum(1 + len(t[4]) for t in tasks[:ncores])
    allc = tmpln * g.n / tn
    return dict(value=allc, unit="template-samples/s", cores=ncores, kind="oracle",
                sample=f"segment 0 of the batched workload: {ncores} seeded reference groups, each the reference "
                       f"matched filter + FFT reconstruction of {per_group} seeded neighbours (full 2^20-sample "
                       f"series), numpy FP64, one group per core in a process pool ({tn:.2f} s); "
                       f"extrapolated to the workload as samples/s",
                extrapolated=True, cpu_model=model, cores_usable=cores,
                single_core=dict(value=single, templates=tmpl1, seconds=t1), all_core_templates=tmpln,
                all_core_seconds=tn)


def cpu_baseline(w, n_nbr_sample, n_cmp=12):
    """The FP64 oracle on the host: reference matched filter and FFT-based
    reconstruction of a sample of neighbours (full series each).  Beside it,
    the host analogue of the paper's cost comparison (sec. IV): direct matched
    filtering of `n_cmp` neighbours (template generated on the fly, one
    transform each) against the ratio filter for the same neighbours (stored
    kernels, overlap-add convolution with the reference series)."""
    from oracle import mf as omf
    from oracle import ratio as orat
    g = w["grid"]
    nb = w["nbrs"][:n_nbr_sample]
    kern = [orat.build_kernel(g, w["ref"], k) for k in nb]          # build: not timed
    norms = [omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *k)) for k in nb]
    t0 = time.perf_counter()
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *w["ref"])
    t_ref = time.perf_counter() - t0
    for kb, nk in zip(kern, norms):
        orat.reconstruct(zr, kb["m_lo"], kb["taps"], nr / nk)
    dt = time.perf_counter() - t0
    # cost comparison on the first n_cmp neighbours
    t0 = time.perf_counter()
    for k in nb[:n_cmp]:
        omf.grid_snr_series(g, w["xf"], w["psd"], *k)
    t_direct = time.perf_counter() - t0
    t0 = time.perf_counter()
    for kb, nk in zip(kern[:n_cmp], norms[:n_cmp]):
        orat.reconstruct_oa(zr, kb["m_lo"], kb["taps"], nr / nk)
    t_oa = time.perf_counter() - t0
    group = len(w["nbrs"]) + 1
    per_direct = t_direct / n_cmp
    per_ratio = t_oa / n_cmp + t_ref / group        # the reference's filter shared by its group
    return dict(value=(1 + len(nb)) * g.n / dt, unit="template-samples/s", cores=1, kind="oracle",
                sample=f"reference MF + FFT-based reconstruction of {len(nb)} of 256 neighbours, "
                       f"full 2^21-sample series, numpy FP64 on one host core ({dt:.2f} s)",
                ratio_vs_direct=dict(templates=n_cmp, direct_s_per_template=per_direct,
                                     ratio_s_per_template=per_ratio, reference_mf_s=t_ref,
                                     cost_reduction=1.0 - per_ratio / per_direct,
                                     note="host, one core: direct = template spectrum + inverse FFT; ratio = "
                                          "overlap-add convolution of the reference series with the stored "
                                          "kernel, reference filter shared by the 257-template group"))


def headline_leg(dev, steps, warmup, cache_path=None):
    """The headline step at the batched workload's full shape (8 x 256 s at
    4096 Hz, 64 references, 10,136 kernels): one rf_batch_run per step, timed
    over exactly `steps` runs after `warmup`, with the reconstruction graph's
    duration (persistent launch + read-out) from the library's HIP events on
    the batch's stream, every step."""
    log("bench: generating the batched workload (8 x 256 s, 64 references)")
    wb = synth.workload_batched()
    g = wb["grid"]
    nseg = len(wb["segments"])
    stream = torch.cuda.Stream(dev)
    ctx = rf.Context(0, stream)
    psd = torch.from_numpy(wb["psd"]).to(dev)
    xf = torch.from_numpy(np.stack(wb["segments"])).to(dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        ksets = [rf.ratio_kernel_build(ctx, g, psd, r, grp) for r, grp in zip(wb["refs"], wb["groups"])]
        stream.synchronize()
        t_build = time.perf_counter() - t0
        batch = rf.Batch(ctx, g, psd, wb["refs"], ksets, nseg=nseg)
        t0 = time.perf_counter()
        chunks = batch.autotune(xf, cache_path)
        t_tune = time.perf_counter() - t0
        tuning = batch.tuning()
        lens = np.concatenate([k.info()["len"] for k in ksets])
        sum_l = int(lens.sum())
        corr = [k.split_steps(1024) for k in ksets]
        corr_steps, all_steps = sum(c for c, _ in corr), sum(a for _, a in corr)
        ktot = batch.ktotal
        peaks = torch.empty((nseg, ktot, 2), dtype=torch.int32, device=dev)
        trig = torch.empty((1 << 20, 5), dtype=torch.int32, device=dev)
        rec = []

        def step():
            out = batch.run(xf, 6.0, trig_cap=1 << 20, peaks=peaks, trig=trig)
            rec.append(batch.last_recon_ms())
            return out

        log(f"bench: headline: {ktot} kernels ({lens.min()}..{lens.max()} taps), tuning {tuning} "
            f"(autotune {t_tune:.2f} s); "
            f"{warmup} warm-up + {steps} timed steps")
        for _ in range(warmup):
            step()
        cap0, rep0 = batch.graph_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            last = step()
            log(f"bench: headline step {i + 1}/{steps}: reconstruction {rec[-1]:.1f} ms")
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        cap1, rep1 = batch.graph_stats()
    vals, idx = rf.decode_peaks(peaks.view(nseg * ktot, 2))
    trig_list = rf.decode_triggers(trig, last["ntrig"])
    # each segment's injection recovered by its template's series at the injection time
    found = 0
    for (s_, m1, m2, snr, t0_, phi) in wb["injections"]:
        found += any(t[1] == s_ and abs(t[2] - int(round(t0_ * g.fs))) <= 8 for t in trig_list)
    res = dict(wb=wb, grid=g, nseg=nseg, ktot=ktot, nref=len(wb["refs"]), lens=lens, sum_l=sum_l,
               corr_frac=corr_steps / max(all_steps, 1), exec_taps=all_steps * 16 * 32, chunks=chunks, tuning=tuning,
               wall_ms=wall, recon_ms=rec[-steps:], build_s=t_build, tune_s=t_tune,
               captures_in_timed=cap1 - cap0, replays_in_timed=rep1 - rep0, ntrig=last["ntrig"],
               peak_max=float(vals.max()), injections_found=found)
    batch.free()
    for k in ksets:
        k.free()
    ctx.close()
    del peaks, trig, xf
    return res


def batched_leg(dev):
    """Reduced batched uneven workload (4 segments of 32 s at 1024 Hz, 8
    references with 8..96 lattice neighbours, autotuned chunks): one persistent
    split-FP16 launch in captured graphs, replays only, against the
    per-(segment, reference) call loop on the same data."""
    wb = synth.workload_batched(n_seg=4, n_ref=8, duration=32.0, fs=1024.0, f_low=25.0, seed=1003,
                                nbr_range=(8, 96))
    g = wb["grid"]
    stream = torch.cuda.Stream(dev)
    ctx = rf.Context(0, stream)
    psd = torch.from_numpy(wb["psd"]).to(dev)
    xf = torch.from_numpy(np.stack(wb["segments"])).to(dev)
    nseg = len(wb["segments"])
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        ksets = [rf.ratio_kernel_build(ctx, g, psd, r, grp) for r, grp in zip(wb["refs"], wb["groups"])]
        batch = rf.Batch(ctx, g, psd, wb["refs"], ksets, nseg=nseg)
        chunks = batch.autotune(xf)
        tuning = batch.tuning()
        sum_l = sum(sum(k.info()["len"]) for k in ksets)
        peaks = torch.empty((nseg, batch.ktotal, 2), dtype=torch.int32, device=dev)
        trig = torch.empty((1 << 20, 5), dtype=torch.int32, device=dev)
        batch.run(xf, 6.0, trig_cap=1 << 20, peaks=peaks, trig=trig)          # capture
        stream.synchronize()
        cap0, _ = batch.graph_stats()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            out = batch.run(xf, 6.0, trig_cap=1 << 20, peaks=peaks, trig=trig)
        t_batch = (time.perf_counter() - t0) / reps
        cap1, _ = batch.graph_stats()
        z = torch.empty((1, g.n), dtype=torch.complex64, device=dev)

        def loop():
            for s_ in range(nseg):
                for r, K in enumerate(ksets):
                    rf.mf_ref_snr(ctx, g, xf[s_].contiguous(), psd, [wb["refs"][r]], z=z, want_sigma=False)
                    rf.snr_reconstruct(ctx, K, z[0], prec="split16", store=False, fused_thr=6.0)
        loop()
        stream.synchronize()
        t0 = time.perf_counter()
        loop()
        stream.synchronize()
        t_loop = time.perf_counter() - t0
    ktot = batch.ktotal
    flops = 4.0 * g.n * sum_l * nseg
    samples = (ktot + len(wb["refs"])) * g.n * nseg
    res = dict(workload=wb["name"] + "-reduced", segments=nseg, references=len(wb["refs"]),
               kernels=ktot, neighbours_per_ref=[len(x) for x in wb["groups"]], chunks=chunks, tuning=tuning, sum_taps=sum_l,
               batch_ms=t_batch * 1e3, loop_ms=t_loop * 1e3, speedup=t_loop / t_batch,
               graph_captures_while_timed=cap1 - cap0,
               value=samples / t_batch, unit="template-samples/s",
               frac_fp16_peak=flops / t_batch / 1e12 / PEAK_FP16_TFLOPS, ntrig=out["ntrig"])
    batch.free()
    for k in ksets:
        k.free()
    ctx.close()
    return res


def factored_leg(dev, ctx, w, psd, xf, K, steps, tol=2e-6, precs=("split16", "fp32")):
    """Factored reconstruction of the same 256 series through the kernel set's
    leading basis (J FFT correlations + matrix-core mixing), fused read-out,
    series stored; timed like the step for each mixing precision, with its
    error against direct MF."""
    g = w["grid"]
    n = g.n
    nbrs = w["nbrs"]
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = rf.Factored(ctx, K, g, tol=tol, jmax=128)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = F.info()
    J = info["J"]
    zref = torch.empty((1, n), dtype=torch.complex64, device=dev)
    zout = torch.empty((len(nbrs), n), dtype=torch.complex64, device=dev)
    zd, _ = rf.mf_ref_snr(ctx, g, xf, psd, nbrs, want_sigma=False)
    res = dict(J=J, tol=tol, max_resid=float(max(info["resid"])), union_taps=info["len"], build_s=t_build,
               mix_flops=4.0 * J * len(nbrs) * n, fft_transforms=J + 1,
               storage_bytes=dict(basis_spectra_fp32=8 * J * (n // 2), coefficients=4 * J * len(nbrs)))
    for prec in precs:
        rec = []

        def step():
            rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]], z=zref, want_sigma=False)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out = F.reconstruct(zref[0], z_out=zout, fused_thr=6.0, trig_cap=1 << 16, prec=prec)
            b.record(stream)
            rec.append((a, b))
            return out

        log(f"bench: factored {prec}")
        wall, _ = timed(step, steps, 2, stream)
        rms = float(np.mean([a.elapsed_time(b) for a, b in rec[-steps:]]))
        last = step()
        err = (zout - zd).abs().max().item()
        ms = wall / steps
        res[prec] = dict(step_ms=ms, recon_ms=rms, value=(1 + len(nbrs)) * n / (ms * 1e-3),
                         unit="template-samples/s", err_vs_direct_mf=err, ntrig=last["ntrig"])
    del zd
    F.free()
    return res


def ols_leg(dev, ctx, w, psd, xf, K, steps):
    """Blocked frequency-domain (overlap-save) reconstruction of the same 256
    series with the exact truncated kernels, fused read-out, series stored;
    timed like the step, with its error against direct MF."""
    g = w["grid"]
    n = g.n
    nbrs = w["nbrs"]
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    O = rf.Ols(ctx, K, n)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = O.info()
    zref = torch.empty((1, n), dtype=torch.complex64, device=dev)
    zout = torch.empty((len(nbrs), n), dtype=torch.complex64, device=dev)
    rec = []

    def step():
        rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]], z=zref, want_sigma=False)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = O.reconstruct(zref[0], z_out=zout, fused_thr=6.0, trig_cap=1 << 16)
        b.record(stream)
        rec.append((a, b))
        return out

    wall, _ = timed(step, steps, 2, stream)
    rms = float(np.mean([a.elapsed_time(b) for a, b in rec[-steps:]]))
    last = step()
    zd, _ = rf.mf_ref_snr(ctx, g, xf, psd, nbrs, want_sigma=False)
    err = (zout - zd).abs().max().item()
    del zd
    ms = wall / steps
    nb = n // info["hop"]
    parts = sum(info["parts"])
    # per block and kernel: P complex MACs per bin, one 8192-point transform (5 B log2 B flops)
    flops = nb * (parts * info["block"] * 8 + len(nbrs) * 5 * info["block"] * 13)
    res = dict(block=info["block"], hop=info["hop"], partitions_max=info["pmax"], partitions_total=parts,
               spectra_bytes=info["spectra_bytes"], build_s=t_build, step_ms=ms, recon_ms=rms,
               value=(1 + len(nbrs)) * n / (ms * 1e-3), unit="template-samples/s", err_vs_direct_mf=err,
               ntrig=last["ntrig"], fft_mac_flops=flops,
               # against the FP32 vector peak without packed-FP32 instructions (switched off in the build)
               vector_fp32_frac=flops / (rms * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
               vector_fp32_peak_tflops=PEAK_FP32_VECTOR_TFLOPS)
    O.free()
    return res


def bank_leg(dev, ctx, w, psd):
    """Bank organisation (sec. III.A) on a synthetic stochastic 1-3 Msun bank at
    f_low = 20 Hz (stand-in for the paper's minimal-match-0.97 bank): chirp-mass
    bisection to a 10 s duration spread, symmetric-mass-ratio bisection to 500
    templates, median-duration references; then every dependent's ratio kernel
    built on the GPU at the realistic grid (4096 Hz, 2^21 samples, 1e-3 / s)
    for the storage figure (template durations over kernel durations)."""
    g = w["grid"]
    t0 = time.perf_counter()
    bank = synth.stochastic_bank(f0=g.f_low)
    t_place = time.perf_counter() - t0
    t0 = time.perf_counter()
    tau = rf.template_durations(bank, g.f_low)
    grp, refs = rf.bank_organise(bank, tau, max_spread=10.0, max_size=500)
    t_org = time.perf_counter() - t0
    sizes = np.bincount(grp)
    spreads = [float(np.ptp(tau[grp == i])) for i in range(len(refs))]
    dep_tau = 0.0
    dep_taps = 0
    t0 = time.perf_counter()
    for gi, r in enumerate(refs):
        members = [int(i) for i in np.nonzero(grp == gi)[0] if i != r]
        if not members:
            continue
        K = rf.ratio_kernel_build(ctx, g, psd, bank[r], [bank[i] for i in members])
        dep_taps += int(sum(K.info()["len"]))
        dep_tau += float(tau[members].sum())
        K.free()
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    kernel_s = dep_taps / g.fs
    return dict(templates=len(bank), groups=len(refs), group_size_min=int(sizes.min()),
                group_size_median=float(np.median(sizes)), group_size_max=int(sizes.max()),
                duration_spread_max_s=max(spreads), template_duration_s=dict(min=float(tau.min()),
                                                                             max=float(tau.max())),
                placement_s=t_place, organise_s=t_org, kernel_build_s=t_build, dependents=len(bank) - len(refs),
                storage_ratio_dependents=dep_tau / kernel_s, storage_ratio_bank=float(tau.sum()) / kernel_s,
                kernel_taps_total=dep_taps)


def factored_batched_leg(dev, max_set=256, tol=2e-6):
    """The factored form at the batched workload's full shape (8 x 256 s at
    4096 Hz, 64 references, 10,136 kernels): each reference's neighbours in sets
    of at most 256 consecutive lattice points, each set with its own basis
    (kernel and basis builds timed apart); per segment and reference, the
    reference matched filter and the factored reconstruction of every set with
    the fused read-out (series not stored), timed as per-call loop and as one
    batched call (whose peaks must equal the loop's).  The peaks of every series
    are compared with direct matched filtering of the same templates (read-out
    in the transform), which is timed over the same segments."""
    wb = synth.workload_batched()
    g = wb["grid"]
    nseg = len(wb["segments"])
    stream = torch.cuda.current_stream(dev)
    ctx = rf.Context(0, stream)
    psd = torch.from_numpy(wb["psd"]).to(dev)
    xf = torch.from_numpy(np.stack(wb["segments"])).to(dev)
    zref = torch.empty((1, g.n), dtype=torch.complex64, device=dev)
    jvals, resid = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_ref = []                     # per reference: its sets (kernels, basis)
    for r, (ref, grp) in enumerate(zip(wb["refs"], wb["groups"])):
        sets = []
        for a in range(0, len(grp), max_set):
            K = rf.ratio_kernel_build(ctx, g, psd, ref, list(grp[a:a + max_set]))
            F = rf.Factored(ctx, K, g, tol=tol, jmax=128)
            inf = F.info()
            jvals.append(inf["J"])
            resid.append(max(inf["resid"]))
            sets.append((K, F))
        per_ref.append(sets)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    # per-(segment, reference) calls: the reference matched filter, then each set
    pk = [[None] * len(wb["refs"]) for _ in range(nseg)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(nseg):
        for r, ref in enumerate(wb["refs"]):
            rf.mf_ref_snr(ctx, g, xf[s_], psd, [ref], z=zref, want_sigma=False)
            pk[s_][r] = [F.reconstruct(zref[0], store=False, fused_thr=6.0, trig_cap=1 << 18)["peaks"]
                         for K, F in per_ref[r]]
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    # the same in one call (every segment and set, one synchronisation)
    all_sets = [F for sets in per_ref for K, F in sets]
    all_refs = [ref for ref, sets in zip(wb["refs"], per_ref) for _ in sets]
    rf.factored_batch(ctx, g, xf, psd, all_sets, all_refs, 6.0, trig_cap=1 << 18)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bo = rf.factored_batch(ctx, g, xf, psd, all_sets, all_refs, 6.0, trig_cap=1 << 18)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    bv, bi = rf.decode_peaks(bo["peaks"].view(-1, 2))
    cv = np.concatenate([np.concatenate([rf.decode_peaks(p)[0] for p in pk[s_][r]])
                         for s_ in range(nseg) for r in range(len(wb["refs"]))])
    batch_equal = bool(np.array_equal(bv, cv))
    # direct matched filtering of the same templates, and the peaks against it
    t_direct, err, nser = 0.0, 0.0, 0
    for r, grp in enumerate(wb["groups"]):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dpk = [rf.mf_snr_peaks(ctx, g, xf[s_], psd, list(grp), 6.0, trig_cap=1 << 18)["peaks"] for s_ in range(nseg)]
        torch.cuda.synchronize()
        t_direct += time.perf_counter() - t0
        for s_ in range(nseg):
            fv = np.concatenate([rf.decode_peaks(p)[0] for p in pk[s_][r]])
            dv = rf.decode_peaks(dpk[s_])[0]
            err = max(err, float(np.abs(fv - dv).max()))
            nser += len(grp)
    for sets in per_ref:
        for K, F in sets:
            F.free()
            K.free()
    ktot = sum(len(x) for x in wb["groups"])
    samples = (ktot + len(wb["refs"])) * g.n * nseg
    ctx.close()
    return dict(workload=f"batched-{nseg}seg-256s-4096Hz-{len(wb['refs'])}ref-{ktot}kernels", sets=len(jvals),
                J_min=min(jvals), J_max=max(jvals), J_mean=float(np.mean(jvals)), resid_max=float(max(resid)),
                build_s=t_build, recon_s=t_rec, value=samples / t_rec, unit="template-samples/s",
                batch_s=t_batch, batch_value=samples / t_batch, batch_peaks_equal_per_call=batch_equal,
                direct_s=t_direct, direct_value=samples / t_direct, series_checked=nser,
                peak_err_vs_direct=err, within_2e_4=err <= 2e-4,
                note="recon_s: per-(segment, reference) calls (reference MF + factored reconstruction of each "
                     "set); batch_s: every segment and set in one snr_reconstruct_factored_batch call")


def stress_leg(dev, ctx):
    """Next-generation-detector shape: 2048 s at 4096 Hz (2^23 samples), f_low
    10 Hz, 4 references x 1024 lattice neighbours (kernels of 10.8k-67k taps).
    Per reference: its matched filter + fused split-FP16 reconstruction of the
    1024 series (peaks and triggers, series not stored: 4096 x 2^23 complex64
    would be 275 GB), against direct FFT matched filtering of the same 4096
    templates with the same read-out, the blocked frequency-domain form and the
    factored form (one 1024-kernel set per reference, its basis up to 512
    vectors, peaks checked against direct matched filtering); kernel builds
    timed apart.  The learned
    kernels are not used here: a surrogate trained at f_low = 20 Hz does not
    transfer to this band (every kernel would take the exact fallback)."""
    w = synth.workload_stress()
    g = w["grid"]
    psd = torch.from_numpy(w["psd"]).to(dev)
    xf = torch.from_numpy(w["xf"]).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ksets = [rf.ratio_kernel_build(ctx, g, psd, r, grp) for r, grp in zip(w["refs"], w["groups"])]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    lens = np.concatenate([k.info()["len"] for k in ksets])
    zref = torch.empty((1, g.n), dtype=torch.complex64, device=dev)

    def ratio():
        for r, K in zip(w["refs"], ksets):
            rf.mf_ref_snr(ctx, g, xf, psd, [r], z=zref, want_sigma=False)
            rf.snr_reconstruct(ctx, K, zref[0], prec="split16", store=False, fused_thr=6.0, trig_cap=1 << 18)

    zb = torch.empty((128, g.n), dtype=torch.complex64, device=dev)

    def direct():
        for grp, r in zip(w["groups"], w["refs"]):
            rf.mf_snr_peaks(ctx, g, xf, psd, [r] + list(grp), 6.0, trig_cap=1 << 18)

    plans = [rf.Ols(ctx, K, g.n) for K in ksets]

    def ols():
        for r, O in zip(w["refs"], plans):
            rf.mf_ref_snr(ctx, g, xf, psd, [r], z=zref, want_sigma=False)
            O.reconstruct(zref[0], store=False, fused_thr=6.0, trig_cap=1 << 18)

    stream = torch.cuda.current_stream(dev)
    log("bench: stress: overlap-save form")
    ols()
    t_ols, _ = timed(ols, 1, 0, stream)
    pmax = max(O.info()["pmax"] for O in plans)
    for O in plans:
        O.free()
    log("bench: stress: dense split-FP16 reconstruction")
    ratio()
    t_ratio, _ = timed(ratio, 1, 0, stream)
    log("bench: stress: direct matched filtering")
    direct()
    t_direct, _ = timed(direct, 1, 0, stream)
    # peaks of every neighbour by direct matched filtering (untimed), for the factored form's check
    pk_direct = []
    for grp in w["groups"]:
        for a in range(0, len(grp), 128):
            part = list(grp[a:a + 128])
            rf.mf_ref_snr(ctx, g, xf, psd, part, z=zb, want_sigma=False)
            pk_direct.append(rf.decode_peaks(rf.snr_peaks(ctx, zb[:len(part)], 1e9)["peaks"])[0])
    pk_direct = np.concatenate(pk_direct)
    # factored form: each reference's 1024 neighbours form one set with its own basis (up to
    # 512 vectors); sets are built, run and freed one reference at a time (the basis
    # correlations of a set take J x 64 MiB)
    t_fbuild = t_fact = 0.0
    fpk, jinfo = [], []
    for r, grp in zip(w["refs"], w["groups"]):
        log(f"bench: stress: factored set of reference {r}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = rf.Factored(ctx, ksets[w["refs"].index(r)], g, tol=2e-6, jmax=512)
        torch.cuda.synchronize()
        t_fbuild += time.perf_counter() - t0
        jinfo.append(F.info())
        rf.mf_ref_snr(ctx, g, xf, psd, [r], z=zref, want_sigma=False)
        o = F.reconstruct(zref[0], store=False, fused_thr=6.0, trig_cap=1 << 18)     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rf.mf_ref_snr(ctx, g, xf, psd, [r], z=zref, want_sigma=False)
        o = F.reconstruct(zref[0], store=False, fused_thr=6.0, trig_cap=1 << 18)
        torch.cuda.synchronize()
        t_fact += time.perf_counter() - t0
        fpk.append(rf.decode_peaks(o["peaks"])[0])
        F.free()
    fact = dict(sets=len(jinfo), J_min=min(i["J"] for i in jinfo), J_max=max(i["J"] for i in jinfo),
                resid_max=float(max(max(i["resid"]) for i in jinfo)), build_s=t_fbuild, ms=t_fact * 1e3,
                value=(len(lens) + len(w["refs"])) * g.n / t_fact,
                peak_err_vs_direct=float(np.abs(np.concatenate(fpk) - pk_direct).max()))
    fact["within_2e-4"] = fact["peak_err_vs_direct"] <= 2e-4
    ntpl = len(lens) + len(w["refs"])
    samples = ntpl * g.n
    flops = 4.0 * g.n * float(lens.sum())
    res = dict(templates=ntpl, kernel_taps_min=int(lens.min()), kernel_taps_max=int(lens.max()),
               kernel_build_s=t_build, ratio_ms=t_ratio, direct_ms=t_direct,
               ratio_value=samples / (t_ratio * 1e-3), direct_value=samples / (t_direct * 1e-3),
               ols_ms=t_ols, ols_value=samples / (t_ols * 1e-3), ols_partitions_max=pmax,
               unit="template-samples/s", recon_tflops=flops / (t_ratio * 1e-3) / 1e12,
               recon_fp16_frac=flops / (t_ratio * 1e-3) / 1e12 / PEAK_FP16_TFLOPS, factored=fact)
    del zb, zref
    for K in ksets:
        K.free()
    return res


SWEEP_MC = (0.871, 1.219, 1.741, 2.612)
SWEEP_Q = (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0)
SWEEP_THR = (1.0, 3e-1, 1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5)


def sweep_leg(dev, ctx):
    """SNR loss against kernel length (sec. II.D, Fig. 3, and appendix B on the
    chirp mass): for each chirp mass and mass ratio, one injection at
    SNR 20 in coloured noise (512 s, 4096 Hz, f_low 20 Hz); reference of the
    same chirp mass at q = 0.6; the target's kernel truncated at each
    threshold; loss = |peak |z| reconstructed - peak |z| direct| / direct,
    against tau_ratio / tau_target (kernel taps / fs over tau(f_low))."""
    out = {}
    for mc in SWEEP_MC:
        rows = []
        for q in SWEEP_Q:
            w = synth.workload_sweep(mc, q)
            g = w["grid"]
            psd = torch.from_numpy(w["psd"]).to(dev)
            xf = torch.from_numpy(w["xf"]).to(dev)
            z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"], w["tgt"]], want_sigma=False)
            zr = z[0].contiguous()
            rho_m = z[1].abs().max().item()
            tau_t = float(rf.template_durations([w["tgt"]], g.f_low)[0])
            for thr in SWEEP_THR:
                K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], [w["tgt"]], thr=thr)
                L = K.info()["len"][0]
                zk = rf.snr_reconstruct(ctx, K, zr, prec="split16")["z"]
                rho_r = zk.abs().max().item()
                K.free()
                rows.append(dict(q=q, thr=thr, taps=L, x=L / g.fs / tau_t, loss=abs(rho_r - rho_m) / rho_m,
                                 rho_direct=rho_m))
            del z, zr, xf, psd
        # where the loss (worst over q) first stays below 1e-4 and 1e-5, in tau_ratio / tau_target
        cross = {}
        for level in (1e-4, 1e-5):
            xs = []
            for q in SWEEP_Q:
                pts = sorted((r["x"], r["loss"]) for r in rows if r["q"] == q)
                ok = [x for i, (x, l) in enumerate(pts) if all(l2 <= level for _, l2 in pts[i:])]
                xs.append(ok[0] if ok else None)
            cross[str(level)] = None if any(x is None for x in xs) else max(xs)
        at_paper = [r for r in rows if r["thr"] == 1e-3]
        out[str(mc)] = dict(rows=rows, x_at_loss=cross, paper_threshold=dict(
            x_min=min(r["x"] for r in at_paper), x_max=max(r["x"] for r in at_paper),
            loss_max=max(r["loss"] for r in at_paper)))
        log(f"bench: sweep Mc {mc}: loss at 1e-3/s <= {out[str(mc)]['paper_threshold']['loss_max']:.2e}, "
            f"x where loss < 1e-5: {cross['1e-05']}")
    return out


def learned_leg(dev, w, psd, xf, K_exact, build_s, steps):
    stream = torch.cuda.Stream(dev)          # training replays a captured graph: not the null stream
    ctx = rf.Context(0, stream)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        res = _learned(dev, ctx, stream, w, psd, xf, K_exact, build_s, steps)
    torch.cuda.synchronize()
    ctx.close()
    return res


def _learned(dev, ctx, stream, w, psd, xf, K_exact, build_s, steps):
    """Learned kernels (C4 shape): a surrogate trained on 20 000 exact kernels of
    random pairs (1-3 Msun, neighbours within 10 lattice steps) built at 4096 Hz,
    f_low = 20 Hz, n = 2^17, on a 32768-tap window; then the realistic
    workload's 256 kernels from the network alone, from projected SVD
    coefficients, and from 16- and 8-bit codes of the coefficients' residual
    against the network's prediction (and, for comparison, plain codes of the
    coefficients at the same widths), each checked on a 64 s noise segment with
    the reference injected at SNR 20 (fallback to the exact FP64 kernel above
    2e-4), with SNR error against
    direct matched filtering, storage, build time and the reconstruction rate
    with the final set of the 16-bit residual form."""
    g = w["grid"]
    nbrs = w["nbrs"]
    n = g.n
    gb = synth.make_grid(g.fs, 1 << 17, g.f_low)
    npair, nomega, window, batch, lr, tsteps = 20000, 128, 32768, 256, 3e-3, 30000
    refs, pn = synth.surrogate_pairs(gb.f_low, npair, seed=4001)
    omega, theta, order = synth.surrogate_random_inputs(4002, npair, nomega, tsteps, batch)
    om = torch.from_numpy(omega).to(dev)
    od = torch.from_numpy(order).to(dev)
    th = torch.from_numpy(theta).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = rf.Surrogate(ctx, gb, refs, pn, window, om, rank=64)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    S.set_params(th)
    t0 = time.perf_counter()
    hist = S.train(od, lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    inf = S.info()
    gc = synth.make_grid(g.fs, 1 << 18, g.f_low)
    psdc = synth.make_psd(gc)
    # check segment: 64 s of noise with the reference injected at SNR 20 (the loudest injection of the
    # workload), so that a kernel passes only if its error stays within the tolerance on a loud signal
    xc = synth.inject(gc, psdc, synth.noise(gc, psdc, seed=4100), *w["ref"], 20.0, 32.0, 0.0)
    chk = (gc, torch.from_numpy(xc).to(dev), torch.from_numpy(psdc).to(dev))
    zref = torch.empty((1, n), dtype=torch.complex64, device=dev)
    rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]], z=zref, want_sigma=False)
    zd, _ = rf.mf_ref_snr(ctx, g, xf, psd, nbrs, want_sigma=False)
    zo = torch.empty((len(nbrs), n), dtype=torch.complex64, device=dev)

    def err_vs_direct(K):
        rf.snr_reconstruct(ctx, K, zref[0], prec="split16", z_out=zo)
        return (zo - zd).abs().amax(dim=1).cpu().numpy()

    res = dict(training_pairs=npair, window_taps=window, basis_rank=64, numerical_rank=inf["numerical_rank"],
               create_s=t_create, train_steps=tsteps, train_batch=batch, train_lr=lr, train_s=t_train,
               train_ms_per_step=t_train / tsteps * 1e3, loss_first=float(hist[0]),
               loss_last100=float(np.mean(hist[-100:])))
    # network coefficients alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    KN, fb, cerr = S.kernels(g, psd, w["ref"], nbrs, check=chk, tol=2e-4)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    cp = S.project(w["ref"], nbrs)
    cn = S.predict(w["ref"], nbrs)
    crel = (torch.linalg.norm(cn - cp, dim=1) / torch.linalg.norm(cp, dim=1)).cpu().numpy()
    e_net = err_vs_direct(KN)
    res["network"] = dict(build_with_check_s=t_net, fallback=int(sum(fb)), fallback_frac=sum(fb) / len(nbrs),
                          check_err_median=float(np.median(cerr)), check_err_max=float(np.max(cerr)),
                          coef_rel_err_median=float(np.median(crel)), coef_rel_err_max=float(np.max(crel)),
                          snr_err_vs_direct_final=float(e_net.max()),
                          note="every failing kernel replaced by the exact FP64 one")
    KN.free()
    # projected SVD coefficients (complex128, no quantisation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    KP, fbp, cerrp = S.kernels(g, psd, w["ref"], nbrs, coeffs=cp, check=chk, tol=2e-4)
    torch.cuda.synchronize()
    t_proj = time.perf_counter() - t0
    e_proj = err_vs_direct(KP)
    res["svd_coefficients"] = dict(build_with_check_s=t_proj, fallback=int(sum(fbp)),
                                   check_err_max=float(np.max(cerrp)), snr_err_vs_direct=float(e_proj.max()))
    KP.free()
    # learned predictive coding: codes of the residual against the network's prediction,
    # against plain codes of the coefficients at the same width
    final = None
    for bits in (16, 8):
        for net in (True, False):
            codes, scales = S.encode(w["ref"], nbrs, bits=bits, network=net)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cd = S.decode(w["ref"], nbrs, codes, scales, network=net)
            KQ, fbq, cerrq = S.kernels(g, psd, w["ref"], nbrs, coeffs=cd, check=chk, tol=2e-4)
            torch.cuda.synchronize()
            t_q = time.perf_counter() - t0
            eq = err_vs_direct(KQ)
            key = f"{'network_residual' if net else 'plain'}_codes_{bits}bit"
            acc = [k for k in range(len(nbrs)) if fbq[k] == 0]
            res[key] = dict(bits=bits, fallback=int(sum(fbq)), fallback_frac=sum(fbq) / len(nbrs),
                            check_err_median=float(np.median(cerrq)), check_err_max=float(np.max(cerrq)),
                            accepted_snr_err_vs_direct_max=float(eq[acc].max()) if acc else None,
                            snr_err_vs_direct_final=float(eq.max()), decode_build_with_check_s=t_q,
                            bytes_per_kernel=2 * 64 * bits // 8 + 4,
                            code_scale_median=float(scales.median().item()))
            if net and bits == 16:
                final = KQ
            else:
                KQ.free()
    # reconstruction rate with the learned final set (ref MF + split-FP16 + fused peaks)
    def step():
        rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]], z=zref, want_sigma=False)
        rf.snr_reconstruct(ctx, final, zref[0], prec="split16", z_out=zo, fused_thr=6.0, trig_cap=1 << 16)

    wall, _ = timed(step, max(2, steps // 2), 1, stream)
    ms = wall / max(2, steps // 2)
    sum_exact = int(sum(K_exact.info()["len"]))
    sum_final = int(sum(final.info()["len"]))
    nb_bank = 28441
    basis_fp32 = 8 * 64 * window
    res.update(
        exact=dict(build_s=build_s, snr_err_vs_direct=float(err_vs_direct(K_exact).max())),
        storage_bytes=dict(exact_taps_fp32=4 * sum_exact, exact_taps_fp64=8 * sum_exact,
                           svd_coefficients_fp32=8 * 64 * len(nbrs),
                           network_residual_codes_16bit=res["network_residual_codes_16bit"]["bytes_per_kernel"] * len(nbrs),
                           basis_fp32=basis_fp32, network_params=4 * rf.N_MLP_PARAMS,
                           note="the basis and the network are shared by every kernel of the surrogate's range"),
        # storage over a bank of the synthetic stand-in's size (kernels of the realistic average length)
        bank_storage_bytes=dict(templates=nb_bank, exact_taps_fp32=4 * nb_bank * sum_exact // len(nbrs),
                                svd_coefficients_fp32=nb_bank * 8 * 64 + basis_fp32,
                                network_residual_16bit=nb_bank * res["network_residual_codes_16bit"]["bytes_per_kernel"]
                                + basis_fp32 + 4 * rf.N_MLP_PARAMS),
        learned_residual16_step_ms=ms, learned_residual16_value=(1 + len(nbrs)) * n / (ms * 1e-3),
        learned_residual16_kernel_taps_sum=sum_final)
    final.free()
    S.free()
    del zd, zo
    return res


def c2_legs(dev, args, legs):
    """The single-reference realistic workload (512 s at 4096 Hz, n = 2^21,
    reference 1.6+1.2 with 256 lattice neighbours) and the legs that use it."""
    stream = torch.cuda.current_stream(dev)
    log("bench: generating the realistic workload (512 s, 256 neighbours)")
    w = synth.workload_realistic()
    g = w["grid"]
    n = g.n
    nbrs = w["nbrs"]
    xf = torch.from_numpy(w["xf"]).to(dev)
    psd = torch.from_numpy(w["psd"]).to(dev)
    ctx = rf.Context(0, stream)

    # ---- kernel build (timed separately; stored once in the method)
    t0 = time.perf_counter()
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], nbrs)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = K.info()
    lens = np.array(info["len"])
    sum_l = int(lens.sum())
    corr_steps, all_steps = K.split_steps(1024)
    exec_taps = all_steps * 16 * 32                 # steps in units of a 32-kernel tile's step
    corr_frac = corr_steps / max(all_steps, 1)      # steps that also take the two correction products
    log(f"bench: kernel build {build_s:.3f} s, taps {lens.min()}..{lens.max()} (sum {sum_l})")

    zref = torch.empty((1, n), dtype=torch.complex64, device=dev)
    zout = torch.empty((len(nbrs), n), dtype=torch.complex64, device=dev)
    res = {}

    def ref_mf():
        rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]], z=zref, want_sigma=False)

    recon_ms = []

    def step(prec="split16"):
        ref_mf()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = rf.snr_reconstruct(ctx, K, zref[0], prec=prec, z_out=zout, fused_thr=6.0, trig_cap=1 << 16)
        b.record(stream)
        recon_ms.append((a, b))
        return out

    if "step" in legs:
        log("bench: timing the step (reference MF + split-FP16 reconstruction + fused peaks)")
        wall, per = timed(lambda: step("split16"), args.steps, args.warmup, stream)
        rec = [a.elapsed_time(b) for a, b in recon_ms[-args.steps:]]
        res["step"] = dict(wall_ms=wall, per_ms=per, recon_ms=float(np.mean(rec)))
        last = step("split16")
        res["ntrig"] = last["ntrig"]
        vals, idx = rf.decode_peaks(last["peaks"])
        res["peak_max"] = float(vals.max())
    if "fp32" in legs:
        log("bench: timing the FP32 reconstruction")
        recon_ms.clear()
        wall, per = timed(lambda: step("fp32"), max(2, args.steps // 2), 1, stream)
        rec = [a.elapsed_time(b) for a, b in recon_ms[-max(2, args.steps // 2):]]
        res["fp32"] = dict(wall_ms=wall, per_ms=per, recon_ms=float(np.mean(rec)))
    if "direct" in legs:
        log("bench: timing direct FFT matched filtering of the same 257 templates")
        allt = [w["ref"]] + list(nbrs)
        zall = torch.empty((len(allt), n), dtype=torch.complex64, device=dev)

        def direct_stored():
            rf.mf_ref_snr(ctx, g, xf, psd, allt, z=zall, want_sigma=False)
            return rf.snr_peaks(ctx, zall, 6.0, trig_cap=1 << 16)

        def direct():
            return rf.mf_snr_peaks(ctx, g, xf, psd, allt, 6.0, trig_cap=1 << 16)

        wall, per = timed(direct, max(2, args.steps // 2), 1, stream)
        wall_s, _ = timed(direct_stored, max(2, args.steps // 2), 1, stream)
        res["direct"] = dict(wall_ms=wall, per_ms=per, stored_wall_ms=wall_s)
        # accuracy of the reconstruction against direct MF, every sample of every series
        step("split16")
        e16 = (zout - zall[1:]).abs().max().item()
        step("fp32")
        e32 = (zout - zall[1:]).abs().max().item()
        res["err_vs_direct"] = dict(split16=e16, fp32=e32)
        # threshold-unit sensitivity: the same 1e-3 read per tap (|w| >= 1e-3) instead
        # of per second (|w| >= 1e-3 / fs); shorter kernels, larger truncation error
        log("bench: kernels thresholded at 1e-3 per tap")
        Kt = rf.ratio_kernel_build(ctx, g, psd, w["ref"], nbrs, thr=1e-3, unit=rf.RF_THR_PER_TAP)
        lt = np.array(Kt.info()["len"])
        ref_mf()
        rf.snr_reconstruct(ctx, Kt, zref[0], prec="split16", z_out=zout)
        et = (zout - zall[1:]).abs().max().item()
        pd = (zout.abs().amax(dim=1) - zall[1:].abs().amax(dim=1)).abs().max().item()
        tau = rf.template_durations(nbrs, g.f_low)
        res["per_tap"] = dict(threshold=1e-3, kernel_taps_min=int(lt.min()), kernel_taps_max=int(lt.max()),
                              kernel_taps_sum=int(lt.sum()), err_vs_direct=et, peak_err_vs_direct=pd,
                              storage_ratio=float(tau.sum()) / (float(lt.sum()) / g.fs),
                              storage_ratio_per_second=float(tau.sum()) / (float(lens.sum()) / g.fs))
        Kt.free()
        del zall
    if "factored" in legs:
        log("bench: factored reconstruction through the kernel-set basis")
        res["factored"] = factored_leg(dev, ctx, w, psd, xf, K, args.steps)
    if "ols" in legs:
        log("bench: blocked frequency-domain (overlap-save) reconstruction")
        res["ols"] = ols_leg(dev, ctx, w, psd, xf, K, args.steps)
    if "bank" in legs:
        log("bench: bank organisation and storage")
        res["bank"] = bank_leg(dev, ctx, w, psd)
    if "learned" in legs:
        log("bench: learned kernels (training, inference, check and fallback)")
        res["learned"] = learned_leg(dev, w, psd, xf, K, build_s, args.steps)
    torch.cuda.synchronize()

    samples = (1 + len(nbrs)) * n
    out = {"workload": w["name"], "n": n, "fs": g.fs, "f_low": g.f_low, "f_high": g.f_high,
           "neighbours": len(nbrs), "threshold_per_s": 1e-3, "kernel_taps_min": int(lens.min()),
           "kernel_taps_max": int(lens.max()), "kernel_taps_sum": sum_l, "kernel_build_s": build_s}
    if "step" in res:
        ms = res["step"]["wall_ms"] / args.steps
        t_rec = res["step"]["recon_ms"] * 1e-3
        ach = 4.0 * n * sum_l / t_rec / 1e12
        out.update(step_ms=ms, value=samples / (ms * 1e-3), unit="template-samples/s",
                   recon_split16_ms=res["step"]["recon_ms"], ntrig=res.get("ntrig"), peak_max_absz=res.get("peak_max"),
                   roofline={"bound": "mfma", "achieved": ach, "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
                             "frac": ach / PEAK_FP16_TFLOPS, "traffic": counter_traffic("k_recon_f16"),
                             "kernel": "k_recon_f16 (split-FP16 reconstruction)",
                             "executed_over_useful_taps": exec_taps / sum_l, "correction_step_frac": corr_frac,
                             "executed_frac_of_peak": (1 + 2 * corr_frac) * 4.0 * n * exec_taps / t_rec / 1e12
                             / PEAK_FP16_TFLOPS})
    if "fp32" in res:
        t32 = res["fp32"]["recon_ms"] * 1e-3
        out["recon_fp32_ms"] = res["fp32"]["recon_ms"]
        out["fp32_path_value"] = samples / (res["fp32"]["wall_ms"] / max(2, args.steps // 2) * 1e-3)
        out["fp32_roofline_frac"] = 4.0 * n * sum_l / t32 / 1e12 / PEAK_FP32_TFLOPS
    if "direct" in res:
        dms = res["direct"]["wall_ms"] / max(2, args.steps // 2)
        out["direct_fft_mf_ms"] = dms
        out["direct_fft_mf_value"] = samples / (dms * 1e-3)
        # the same filtering with the series stored and read out by a separate kernel
        out["direct_fft_mf_stored_ms"] = res["direct"]["stored_wall_ms"] / max(2, args.steps // 2)
        # HBM roofline on the algorithmic 16 B per template-sample: the template spectrum is
        # formed on chip and the series read out on chip, but a transform of 2^21 points does
        # not fit on chip, so its intermediate is written and read once (8 B each)
        out["direct_fft_mf_roofline"] = {"bound": "hbm", "bytes_per_template_sample": 16,
                                         "achieved": 16 * samples / (dms * 1e-3) / 1e9,
                                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                         "frac": 16 * samples / (dms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                         "traffic": counter_traffic("mf_snr_peaks")}
        out["err_vs_direct_mf"] = res["err_vs_direct"]
        out["threshold_per_tap"] = res["per_tap"]
    for key in ("factored", "ols", "bank", "learned"):
        if key in res:
            out[key] = res[key]
    if "cpu" in legs:
        log("bench: CPU oracle on the realistic workload (one core) and the host cost comparison")
        out["cpu_oracle_one_core"] = cpu_baseline(w, args.cpu_nbrs)
    K.free()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--cpu-nbrs", type=int, default=24)
    ap.add_argument("--only", default="",
                    help="comma list of legs: headline (the batched workload at full shape), and on the "
                         "realistic workload step,fp32,direct,factored,ols,bank,learned, then batched (reduced), "
                         "factored_batched, stress (default: all of these); sweep only when named")
    ap.add_argument("--tuning-cache", default=None,
                    help="launch-settings cache of the headline batch (read if it holds this shape, else "
                         "appended after autotuning), so that profiled runs take the timed run's settings")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-GPU workload is independent; see the sharding design).", file=sys.stderr)
        sys.exit(2)
    legs = set(args.only.split(",")) if args.only else {"headline", "step", "fp32", "direct", "factored", "ols",
                                                        "bank", "batched", "factored_batched", "learned", "stress"}
    if not args.no_cpu:
        legs.add("cpu")
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
           "data": "synthetic"}
    extra = {}
    h = None
    if "headline" in legs:
        h = headline_leg(dev, args.steps, args.warmup, args.tuning_cache)
        g = h["grid"]
        samples = (h["ktot"] + h["nref"]) * g.n * h["nseg"]
        ms = h["wall_ms"] / args.steps
        t_rec = float(np.mean(h["recon_ms"])) * 1e-3
        alg = 4.0 * g.n * h["sum_l"] * h["nseg"]          # complex x real MAC per kept tap and output sample
        ach = alg / t_rec / 1e12
        out.update(value=samples / (ms * 1e-3), unit="template-samples/s", ms_per_step=ms)
        cq = counter_summary("k_recon_f16_queue")
        out["roofline"] = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / PEAK_FP16_TFLOPS,
                           "traffic": None if cq is None else float(cq["traffic_bytes_per_dispatch"]),
                           # the launch settings the counters were taken at (traffic depends on them;
                           # the run's own are config.tuning)
                           "traffic_tuning": None if cq is None else cq.get("tuning"),
                           "kernel": "k_recon_f16_queue (persistent split-FP16 reconstruction, fused read-out)",
                           "kernel_ms": t_rec * 1e3, "flops_per_launch": alg,
                           "timed": "reconstruction graph per step (persistent launch + peak finalisation), "
                                    "HIP events on the batch's stream",
                           "executed_over_useful_taps": h["exec_taps"] / h["sum_l"],
                           "correction_step_frac": h["corr_frac"],
                           "executed_frac_of_peak": (1 + 2 * h["corr_frac"]) * 4.0 * g.n * h["exec_taps"] * h["nseg"]
                           / t_rec / 1e12 / PEAK_FP16_TFLOPS}
        out["config"] = {"workload": f"batched-{h['nseg']}seg-256s-4096Hz-{h['nref']}ref-{h['ktot']}kernels",
                         "segments": h["nseg"], "n": g.n, "fs": g.fs, "f_low": g.f_low, "f_high": g.f_high,
                         "references": h["nref"], "kernels": h["ktot"], "threshold_per_s": 1e-3,
                         "kernel_taps_min": int(h["lens"].min()), "kernel_taps_max": int(h["lens"].max()),
                         "kernel_taps_sum": h["sum_l"], "chunks": h["chunks"], "tuning": h["tuning"],
                         "precision": "split fp16 hi/lo, hi*lo + lo*hi where large taps, fp32 accumulation"}
        extra["headline"] = {"kernel_build_s": h["build_s"], "autotune_s": h["tune_s"],
                             "recon_ms_per_step": h["recon_ms"], "graph_captures_while_timed": h["captures_in_timed"],
                             "graph_replays_while_timed": h["replays_in_timed"], "ntrig": h["ntrig"],
                             "peak_max_absz": h["peak_max"], "injections_with_trigger": h["injections_found"]}
    c2 = {"step", "fp32", "direct", "factored", "ols", "bank", "learned"} & legs
    if c2:
        extra["realistic"] = c2_legs(dev, args, legs)
        if h is None and "value" in extra["realistic"]:
            r = extra["realistic"]
            out.update(value=r["value"], unit=r["unit"], ms_per_step=r["step_ms"], roofline=r["roofline"])
            out["config"] = {"workload": r["workload"], "n": r["n"], "neighbours": r["neighbours"]}
    if "batched" in legs:
        log("bench: batched uneven workload (reduced)")
        extra["batched_reduced"] = batched_leg(dev)
    if "factored_batched" in legs:
        log("bench: factored form at the batched workload's full shape")
        extra["factored_batched"] = factored_batched_leg(dev)
    if "stress" in legs:
        log("bench: next-generation-detector shape (4 x 1024 templates, 2^23 samples)")
        ctx = rf.Context(0, torch.cuda.current_stream(dev))
        extra["stress"] = stress_leg(dev, ctx)
        ctx.close()
    if "sweep" in legs:
        log("bench: SNR loss against kernel length")
        ctx = rf.Context(0, torch.cuda.current_stream(dev))
        extra["sweep"] = sweep_leg(dev, ctx)
        ctx.close()
    torch.cuda.synchronize()
    out["extra"] = extra
    if "cpu" in legs and h is not None:
        log("bench: CPU oracle baseline (seeded subset of the batched workload)")
        out["cpu_baseline"] = cpu_baseline_batched(h["wb"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
