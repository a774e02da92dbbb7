"""Benchmark of the oblivious map on one MI355X.

Workload (plain OMAP, N=2^24): distinct uint64 keys, 64-byte values, built
once, then 2^20 commands in batches of 4096 (Zipf 0.99 over the present keys
with 5 % absent keys, 90 % GET / 10 % PUT).  A step is one pass of the whole
path: the oblivious build of the N pairs, then every batch of the stream.
Inputs sit in HBM before the timed region starts.

The observable store is pinned host memory reached over the host link (the
paper's setting: the store lives off the package); the same workload is also
run with the store in a designated device buffer and reported beside it.

The timed region runs without per-kernel events (they cost about a third of
a batch).  One further step of the same workload on a map created with
BOLT_F_TIMING records HIP events on the launch stream around every kernel;
kernel durations, algorithmic GB/s and the roofline come from that step.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--observable host|device]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
LINK_PEAK_GBS = 64.0    # PCIe 5.0 x16, per direction
PEAKS = {"hbm": HBM_PEAK_GBS, "host_link": LINK_PEAK_GBS, "host_link_duplex": 2 * LINK_PEAK_GBS}

# Share of a batch's page send that the next batch's fetch writes, for a plain
# map: the library's other kernels carry slices (in 64ths: the batch's own
# finish 1, the next dedup 4, resolve 2, place 4 and rebuild 8).  A sealed
# map's fetch writes all of it.  tests/test_bench_host.py checks these
# against the library's source.
SEND_SLICES_64 = {"finish": 1, "group": 2, "resolve": 1, "place": 3, "compose": 6}
FETCH_SEND_FRACTION = (64 - sum(SEND_SLICES_64.values())) / 64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(cls, sz, n, npad, n_ops, host_roles, send_share=0.0):
    """Algorithmic bytes of ONE launch of a kernel class on the resource that
    bounds it.  `send_share` is the fraction of the previous batch's rebuilt
    pages that an average fetch launch writes (pinned store, batches of 256
    commands or more): those launches use both directions of the link.

    sort passes (HBM): read + write every 8-byte tag, 16 B x npad.
    expansion passes (HBM): read + write every 8-byte slot, 16 B x B*Z.
    page write-out: the M observable pages written once (host link in host
      mode); in device mode also the K HBM bins, the N keys + values and the
      B*Z slots read (HBM).
    fetch, per batch: the observable pages read, about 2 (1 - alpha) per
      command (host link), plus the previous batch's pages written when it
      carries their send (both directions of the link); in device mode both
      whole bins of every command.
    send on its own (flush), per batch: every observable page read is
      written back once (host link); in device mode also read from the outbox.
    rebuild (compose), per batch: each page read is read from the stage and
      written to the outbox (HBM).
    """
    pb, B, Z, K, M, vs = sz["page_bytes"], sz["B"], sz["Z"], sz["K"], sz["M"], sz["vs"]
    host = sz["host"]
    if cls in ("sort_global", "sort_tile", "sort_merge"):
        return 16 * npad, "hbm"
    if cls == "expand":
        return 16 * B * Z, "hbm"
    if cls == "page_writeout":
        if host:
            return M * pb, "host_link"
        return B * pb + n * (8 + vs) + B * Z * 8, "hbm"
    if cls == "acc_fetch":
        if not host:
            return 2 * n_ops * pb, "hbm"
        return (host_roles * pb * (1 + send_share), "host_link_duplex" if send_share else "host_link")
    if cls == "acc_ship":
        return (host_roles * pb, "host_link") if host else (2 * host_roles * pb, "hbm")
    if cls == "acc_compose":
        return 2 * host_roles * pb, "hbm"
    return None, None


def run_mode(args, wl, dev_t, B, torch, observable, seal=False, decomposed=False):
    n, vs = wl.n, wl.vs
    d_keys, d_vals, d_ops, d_qk, d_qv, d_out, d_st, bounds = dev_t
    obs = B.BOLT_OBS_HOST_PINNED if observable == "host" else B.BOLT_OBS_DEVICE
    p = B.params(wl.cap, vs, observable=obs)
    if args.graphs:
        p.flags |= B.BOLT_F_GRAPHS
    if seal:
        p.flags |= B.BOLT_F_SEAL
    if decomposed:
        p.flags |= B.BOLT_F_DECOMPOSED
    sz = B.sizes_of(p)
    sz["vs"] = vs
    sz["host"] = observable == "host"
    stream = torch.cuda.current_stream()
    nsteps = args.warmup + args.steps
    t0 = time.time()
    maps = [B.Map(p) for _ in range(nsteps)]
    pt = B.params(wl.cap, vs, observable=obs)
    pt.flags |= B.BOLT_F_TIMING | (B.BOLT_F_SEAL if seal else 0) | (B.BOLT_F_DECOMPOSED if decomposed else 0)
    tmap = B.Map(pt)
    torch.cuda.synchronize()
    log("[%s] created %d maps (%.1fs); footprint hbm=%.2f GiB obs=%.2f GiB" % (
        observable, nsteps + 1, time.time() - t0, B.footprint(p)[0] / 2**30, B.footprint(p)[1] / 2**30))
    nb = len(bounds) - 1

    def run_step(m):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 2)]
        evs[0].record(stream)
        B.check(m.build(d_keys, d_vals), "bolt_build")
        evs[1].record(stream)
        for bi in range(nb):
            a, b = int(bounds[bi]), int(bounds[bi + 1])
            B.check(m.access(d_ops[a:b], d_qk[a:b], d_qv[a:b], d_out[a:b], d_st[a:b]), "bolt_access_batch")
            if bi == nb - 1:  # the last batch's rebuilt pages reach the store inside the step
                B.check(m.flush(), "bolt_flush")
            evs[bi + 2].record(stream)
        return evs

    for w in range(args.warmup):
        run_step(maps[w])
        B.check(maps[w].status(), "warmup status")
        maps[w].close()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_events = [run_step(maps[args.warmup + s]) for s in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    build_ms, query_ms, lat = [], [], []
    for evs in step_events:
        build_ms.append(evs[0].elapsed_time(evs[1]))
        query_ms.append(evs[1].elapsed_time(evs[-1]))
        lat.extend(evs[i].elapsed_time(evs[i + 1]) for i in range(1, len(evs) - 1))
    for s in range(args.steps):
        B.check(maps[args.warmup + s].status(), "status")
    st = maps[-1].stats()
    log("[%s] step stats: %s" % (observable, st))
    if not (d_st.cpu().numpy()[d_ops.cpu().numpy() == 0] <= 1).all():
        raise SystemExit("bad GET status")

    # instrumented step: per-kernel HIP events on the launch stream
    run_step(tmap)
    B.check(tmap.status(), "status")
    times = tmap.kernel_times()
    tmap.close()

    # plain per-call form: one command per call, on the last map
    m = maps[-1]
    kpc = min(args.per_call, int(bounds[-1]))
    if kpc:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(kpc + 1)]
        one = [(d_ops[i:i + 1], d_qk[i:i + 1], d_qv[i:i + 1], d_out[i:i + 1], d_st[i:i + 1]) for i in range(kpc)]
        ev[0].record(stream)
        for i in range(kpc):
            B.check(m.access(*one[i], stream=stream), "per-call")
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        pc_lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(kpc)]
        pc_ops = kpc / (ev[0].elapsed_time(ev[-1]) / 1e3)
        B.check(m.status(), "status")
    for mm in maps:
        mm.close()

    K = args.steps
    n_ops = int(bounds[-1])
    npad = 1
    while npad < n:
        npad <<= 1
    host_roles = 2 * n_ops * sz["M"] / sz["B"]  # about 2 (1 - alpha) observable pages per command
    kernels = {}
    for cls, (cnt, ms) in sorted(times.items(), key=lambda kv: -kv[1][1]):
        if cnt == 0:
            continue
        ent = {"launches": cnt, "total_ms": round(ms, 3), "avg_us": round(1e3 * ms / cnt, 2)}
        carried = 1.0 if seal else FETCH_SEND_FRACTION
        send_share = carried * (nb - 1) / nb if (sz["host"] and n_ops / nb >= 256) else 0.0
        per, bound = kernel_bytes(cls, sz, n, npad, n_ops / nb, host_roles / nb, send_share)
        if per is not None:
            gbs = per / (ms / cnt / 1e3) / 1e9
            peak = PEAKS[bound]
            ent.update({"bytes_per_launch": int(per), "achieved_GBps": round(gbs, 1), "bound": bound,
                        "frac_of_peak": round(gbs / peak, 4)})
        kernels[cls] = ent
    lat_np = np.array(lat)
    return {
        "ops_per_s": n_ops * K / (sum(query_ms) / 1e3),
        "build_keys_per_s": n * K / (sum(build_ms) / 1e3),
        "build_ms": float(np.mean(build_ms)),
        "query_ms": float(np.mean(query_ms)),
        "ms_per_step": wall * 1e3 / K,
        "lat_p50": float(np.percentile(lat_np, 50)),
        "lat_p99": float(np.percentile(lat_np, 99)),
        "per_call": {"ops_per_s": round(pc_ops, 1), "p50_ms": round(float(np.percentile(pc_lat, 50)), 4),
                     "p99_ms": round(float(np.percentile(pc_lat, 99)), 4), "calls": kpc} if kpc else None,
        "kernels": kernels,
        "sizes": sz,
        "stats": st,
    }


# kernel class -> (kernel in the rocprofv3 counter summary, sources it is built from)
PROFILED = {
    "acc_ship": ("bolt::k_acc_ship", ("k_access.hip", "seal_dev.h", "bolt_dev.h", "bolt_impl.h")),
    "acc_compose": ("bolt::k_acc_compose<false, false>", ("k_access.hip", "seal_dev.h", "bolt_dev.h", "bolt_impl.h")),
    "acc_fetch": ("bolt::k_acc_fetch<false, false>", ("k_access.hip", "seal_dev.h", "bolt_dev.h", "bolt_impl.h")),
    "sort_global": ("bolt::k_bitonic_global<*, false>", ("k_prim.hip", "bolt_dev.h", "bolt_impl.h")),
    "sort_merge": ("bolt::k_bitonic_tile<false>", ("k_prim.hip", "bolt_dev.h", "bolt_impl.h")),
    "page_writeout": ("bolt::k_writeout<false>", ("k_build.hip", "seal_dev.h", "bolt_dev.h", "bolt_impl.h")),
}


def measured_traffic(cls, mode):
    """HBM / fabric bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy calibration) from the committed rocprofv3 counter summary, or None
    when the kernel's sources have changed since the counters were taken."""
    import hashlib

    ent = PROFILED.get(cls)
    path = os.path.join(ROOT, "profiles", "traffic_plain_omap_n24_v64.json")
    if ent is None or not os.path.exists(path):
        return None
    prof = json.load(open(path))
    for fn in ent[1]:
        src = os.path.join(ROOT, "paper_2509_01742_amd", "csrc", fn)
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != prof["sources"].get(fn):
            return None
    kern = prof["modes"].get(mode, {}).get("kernels", {})
    if "*" in ent[0]:  # a kernel with several instantiations: the one launched most
        head, tail = ent[0].split("*")
        names = [nm for nm in kern if nm.startswith(head) and nm.endswith(tail)]
        name = max(names, key=lambda nm: kern[nm]["launches"]) if names else None
    else:
        name = ent[0]
    k = kern.get(name) if name else None
    if k is None:
        return None
    fb, wb = round(k["fetch_bytes"]), round(k["write_bytes"])
    return {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb, "kernel": name, "grid": k["grid"],
            "source": "profiles/traffic_plain_omap_n24_v64.md"}


def roofline_of(res, cls, mode):
    k = res["kernels"].get(cls)
    if not k or "achieved_GBps" not in k:
        return None
    peak = PEAKS[k["bound"]]
    return {"bound": k["bound"], "kernel": cls, "achieved": k["achieved_GBps"], "peak": peak, "unit": "GB/s",
            "frac": round(k["achieved_GBps"] / peak, 4), "traffic": measured_traffic(cls, mode),
            "bytes_per_launch": k["bytes_per_launch"], "avg_launch_us": k["avg_us"], "launches": k["launches"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--ops", type=int, default=1 << 20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--observable", choices=["host", "device"], default="host",
                    help="store of the headline figures (the other mode is reported beside them)")
    ap.add_argument("--single-mode", action="store_true", help="do not run the other observable mode")
    ap.add_argument("--per-call", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-batches", type=int, default=512)
    ap.add_argument("--no-multi", action="store_true", help="skip the 64-map batched figures")
    ap.add_argument("--graphs", action="store_true", help="maps replay captured graphs per batch-size class")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default network schedules")
    ap.add_argument("--no-seal", action="store_true", help="skip the sealed-store figures")
    ap.add_argument("--no-build-heavy", action="store_true", help="skip the N=2^26 build figures (config 3)")
    ap.add_argument("--no-alpha-sweep", action="store_true", help="skip the alpha sweep of the pinned store")
    ap.add_argument("--dynamics", type=int, default=0, metavar="ACCESSES",
                    help="instead of the benchmark: the bound validation of Sec. 4.3 over this many accesses per "
                         "configuration (the paper uses 10^9)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving figures")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="steady window of each open-loop serving run (config 5: 60 s)")
    ap.add_argument("--no-decomposed", action="store_true", help="skip the decomposed-HBM-store figures")
    ap.add_argument("--no-config1", action="store_true", help="skip the N=2^16 per-call figures (config 1)")
    ap.add_argument("--build-heavy-only", action="store_true",
                    help="run only config 3 (the N=2^26 build), for counter profiles")
    ap.add_argument("--multi-only", action="store_true",
                    help="run only config 4 (64 maps in many-map calls against one-map calls), for kernel profiles")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="MiB of a plain device copy run first (scales profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the oblivious map runs on a single MI355X here (sharding across "
              "GPUs is a design note, not an implemented path); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_01742_amd as B
    import synth

    torch.cuda.set_device(0)
    if args.dynamics:
        res = run_dynamics(B, torch, args.dynamics)
        print(json.dumps({"metric": "bound validation (Sec. 4.3): largest bin load, HBM-bin items and stash over a "
                                    "long uniform access stream", "dynamics": res}), flush=True)
        return
    dev = torch.device("cuda:0")
    if args.build_heavy_only:  # config 3 alone (for counter profiles of the N=2^26 build)
        if args.copy_calib:
            src = torch.empty(args.copy_calib << 20, dtype=torch.uint8, device=dev).fill_(1)
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            del src
            log("copy calibration: %d MiB device-to-device" % args.copy_calib)
        heavy = run_build_heavy(B, torch, synth, not args.no_autotune)
        print(json.dumps({"metric": "build keys/s at N=2^26 (config 3)", "build_heavy": heavy}), flush=True)
        return
    if args.multi_only:  # config 4 alone (for kernel profiles of the many-map calls)
        print(json.dumps({"metric": "many-map build keys/s and access ops/s (config 4)",
                          "multi_map": run_multi(B, torch)}), flush=True)
        return
    n = 1 << args.n_log2
    t0 = time.time()
    wl = synth.config2(n=n, n_ops=args.ops, batch=args.batch)
    log("workload %s: n=%d ops=%d batches=%d (%.1fs)" % (wl.name, wl.n, wl.n_ops, len(wl.batches), time.time() - t0))
    ops_all = np.concatenate([b[0] for b in wl.batches])
    keys_all = np.concatenate([b[1] for b in wl.batches])
    vals_all = np.concatenate([b[2] for b in wl.batches])
    dev_t = (torch.from_numpy(wl.build_keys.view(np.int64)).to(dev), torch.from_numpy(wl.build_vals).to(dev),
             torch.from_numpy(ops_all).to(dev), torch.from_numpy(keys_all.view(np.int64)).to(dev),
             torch.from_numpy(vals_all).to(dev), torch.zeros((ops_all.size, wl.vs), dtype=torch.uint8, device=dev),
             torch.zeros(ops_all.size, dtype=torch.uint8, device=dev),
             np.cumsum([0] + [b[0].size for b in wl.batches]))
    if args.copy_calib:
        src = torch.empty(args.copy_calib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: %d MiB device-to-device" % args.copy_calib)

    tuned = None
    if not args.no_autotune:  # schedules of the sort and expansion networks, outside the timed regions
        t0 = time.time()
        B.check(B.autotune(1 << 25), "bolt_autotune")
        torch.cuda.synchronize()
        tuned = {"seconds": round(time.time() - t0, 2), "table": B.tune_table()}
        log("autotune: %.1fs %s" % (tuned["seconds"], [(e["log2_n"], e["sort_tile_log"], e["sort_pass_strides"],
                                                         e["expand_pass_stages"]) for e in tuned["table"]]))
    main_res = run_mode(args, wl, dev_t, B, torch, args.observable)
    other = None
    if not args.single_mode:
        other_mode = "device" if args.observable == "host" else "host"
        o = run_mode(args, wl, dev_t, B, torch, other_mode)
        other = {"observable": other_mode, "ops_per_s": round(o["ops_per_s"], 1),
                 "build_keys_per_s": round(o["build_keys_per_s"], 1),
                 "batch_latency_ms": {"p50": round(o["lat_p50"], 4), "p99": round(o["lat_p99"], 4)},
                 "per_call_ops_per_s": (o["per_call"] or {}).get("ops_per_s"), "kernels": o["kernels"]}

    # the dominant kernel of the headline step (by device time), and the
    # HBM-bound sort pass of the build
    ks = main_res["kernels"]
    dominant = max((c for c in ks if "achieved_GBps" in ks[c]), key=lambda c: ks[c]["total_ms"])
    roofline = roofline_of(main_res, dominant, args.observable)
    roofline_sort = roofline_of(main_res, "sort_global", args.observable)

    sealed = None
    if not args.no_seal:  # the same workload with every observable page sealed (ChaCha20-Poly1305)
        sres = run_mode(args, wl, dev_t, B, torch, args.observable, seal=True)
        sealed = {"observable": args.observable, "ops_per_s": round(sres["ops_per_s"], 1),
                  "build_keys_per_s": round(sres["build_keys_per_s"], 1),
                  "batch_latency_ms": {"p50": round(sres["lat_p50"], 4), "p99": round(sres["lat_p99"], 4)},
                  "relative_to_plain": {"ops": round(sres["ops_per_s"] / main_res["ops_per_s"], 4),
                                        "build": round(sres["build_keys_per_s"] / main_res["build_keys_per_s"], 4)},
                  "kernels": {c: sres["kernels"][c] for c in ("acc_fetch", "acc_compose", "acc_ship", "page_writeout")
                              if c in sres["kernels"]}}
        log("sealed: %s" % json.dumps({k: v for k, v in sealed.items() if k != "kernels"}))
    decomp = None
    if not args.no_decomposed:  # the decomposed HBM store (Sec. 5.2) on the same workload
        dres = run_mode(args, wl, dev_t, B, torch, args.observable, decomposed=True)
        pp = B.params(wl.cap, wl.vs)
        pd = B.params(wl.cap, wl.vs)
        pd.flags |= B.BOLT_F_DECOMPOSED
        decomp = {"observable": args.observable, "ops_per_s": round(dres["ops_per_s"], 1),
                  "build_keys_per_s": round(dres["build_keys_per_s"], 1),
                  "batch_latency_ms": {"p50": round(dres["lat_p50"], 4), "p99": round(dres["lat_p99"], 4)},
                  "relative_to_pages": {"ops": round(dres["ops_per_s"] / main_res["ops_per_s"], 4),
                                        "build": round(dres["build_keys_per_s"] / main_res["build_keys_per_s"], 4)},
                  "hbm_bytes": {"pages": B.footprint(pp)[0], "decomposed": B.footprint(pd)[0]},
                  "config5_admitted_under_budget": serving_admission(B)}
        log("decomposed: %s" % json.dumps(decomp))
    serving = None
    if not args.no_serving:
        serving = run_serving(B, seconds=args.serve_seconds)
        serving["sealed_commands"] = run_serving_sealed(B)
    multi = None
    if not args.no_multi:
        multi = run_multi(B, torch)
        log("multi-map: %s" % json.dumps(multi))
    sweep = None
    if not args.no_alpha_sweep and args.observable == "host":
        sweep = run_alpha_sweep(B, torch, wl, dev_t)
    heavy = None
    if not args.no_build_heavy:
        heavy = run_build_heavy(B, torch, synth, not args.no_autotune)
        log("build-heavy: %s" % json.dumps({k: v for k, v in heavy.items() if k != "phases"}))
    cfg1 = None
    if not args.no_config1:
        cfg1 = run_config1(B, torch, with_oracle=not args.no_cpu_baseline)
        log("config 1: %s" % json.dumps(cfg1))
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_batches)
    sz = main_res["sizes"]
    out = {
        "metric": "oblivious get/put per sec + build keys/s at N=2^24 (1 GPU); p50/p99 latency",
        "value": round(main_res["ops_per_s"], 1),
        "unit": "ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "capacity": wl.cap, "value_bytes": wl.vs,
                   "ops_per_step": int(ops_all.size), "batch": args.batch, "zipf_s": 0.99, "absent_frac": 0.05,
                   "get_frac": 0.9, "observable": args.observable, "c": 8, "alpha": 0.2, "Z": sz["Z"],
                   "page_bytes": sz["page_bytes"]},
        "build_keys_per_s": round(main_res["build_keys_per_s"], 1),
        "build_ms": round(main_res["build_ms"], 3),
        "query_ms": round(main_res["query_ms"], 3),
        "batch_latency_ms": {"p50": round(main_res["lat_p50"], 4), "p99": round(main_res["lat_p99"], 4)},
        "per_call": main_res["per_call"],
        "roofline": roofline,
        "roofline_sort": roofline_sort,
        "kernels": ks,
        "other_observable_mode": other,
        "autotune": tuned,
        "sealed": sealed,
        "decomposed": decomp,
        "multi_map": multi,
        "build_heavy": heavy,
        "alpha_sweep": sweep,
        "serving": serving,
        "config1_per_call": cfg1,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_config1(B, torch, with_oracle=True):
    """Config 1: a map of N=2^16 u64 keys and values, built once, then 2^14
    single GETs (90 % present, 10 % absent) and 2^12 single PUTs over present
    keys.  Per-call form: each command its own call, HIP events between calls
    on the launch stream (latency per command, ops/s over the whole run).
    Batched form: the same commands in order, in batches of 4096, on a fresh
    map.  Every answer of both forms is checked against a dictionary run of
    the commands.  The oracle runs the same commands one call each on the
    host (one thread)."""
    import synth

    wl = synth.config1()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ops = np.concatenate([b[0] for b in wl.batches])
    keys = np.concatenate([b[1] for b in wl.batches])
    vals = np.concatenate([b[2] for b in wl.batches])
    nq = ops.size
    # expected answers: the dictionary semantics, commands in order
    d = {int(k): bytes(v) for k, v in zip(wl.build_keys.tolist(), wl.build_vals)}
    want_st = np.zeros(nq, np.uint8)
    want_v = np.zeros((nq, wl.vs), np.uint8)
    for i in range(nq):
        k = int(keys[i])
        if ops[i] == 0:
            if k in d:
                want_st[i] = 1
                want_v[i] = np.frombuffer(d[k], np.uint8)
        else:
            want_st[i] = 1 if k in d else 2
            d[k] = bytes(vals[i])
    d_keys = torch.from_numpy(wl.build_keys.view(np.int64)).to(dev)
    d_vals = torch.from_numpy(wl.build_vals).to(dev)
    d_ops = torch.from_numpy(ops).to(dev)
    d_qk = torch.from_numpy(keys.view(np.int64)).to(dev)
    d_qv = torch.from_numpy(vals).to(dev)
    out = {"workload": "plain-omap-n16: N=2^16 u64 keys and values, pinned store; 2^14 single GETs (90 %% present, "
                       "10 %% absent) then 2^12 single PUTs over present keys (%d commands), every answer checked "
                       "against a dictionary" % nq}
    for form in ("per_call", "batched"):
        m = B.Map(B.params(wl.n, wl.vs))
        B.check(m.build(d_keys, d_vals), "bolt_build")
        d_out = torch.zeros((nq, wl.vs), dtype=torch.uint8, device=dev)
        d_st = torch.zeros(nq, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        step = 1 if form == "per_call" else 4096
        cuts = list(range(0, nq, step)) + [nq]
        sl = [(d_ops[a:b], d_qk[a:b], d_qv[a:b], d_out[a:b], d_st[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(sl) + 1)]
        ev[0].record(stream)
        for i, a in enumerate(sl):
            B.check(m.access(*a, stream=stream), "config 1 access")
            ev[i + 1].record(stream)
        B.check(m.flush(), "bolt_flush")
        torch.cuda.synchronize()
        B.check(m.status(), "config 1 status")
        if not (np.array_equal(d_st.cpu().numpy(), want_st) and np.array_equal(d_out.cpu().numpy(), want_v)):
            raise SystemExit("config 1: answers differ from the dictionary (%s)" % form)
        total = ev[0].elapsed_time(ev[-1])
        lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(len(sl))])
        out[form] = {"calls": len(sl), "ops_per_s": round(nq / (total / 1e3), 1),
                     "p50_ms": round(float(np.percentile(lat, 50)), 4),
                     "p99_ms": round(float(np.percentile(lat, 99)), 4), "answers_checked": nq}
        m.close()
    out["batched_over_per_call"] = round(out["batched"]["ops_per_s"] / out["per_call"]["ops_per_s"], 2)
    if with_oracle:
        import oracle as O

        t0 = time.perf_counter()
        om = O.OracleMap(wl.n, wl.vs, key=bytes(range(32)))
        assert om.build(wl.build_keys, wl.build_vals) == 0
        t1 = time.perf_counter()
        for b in wl.batches:
            om.access(*b)
        t2 = time.perf_counter()
        out["cpu_oracle"] = {"kind": "oracle", "cores": 1, "build_s": round(t1 - t0, 3), "commands_s": round(t2 - t1, 3),
                             "ops_per_s": round(nq / (t2 - t1), 1),
                             "sample": "the whole config: build of 2^16 keys, then the %d commands one call each" % nq}
    return out


def run_alpha_sweep(B, torch, wl, dev_t, nb_max=64, alphas=(10, 200, 500, 800)):
    """The paper's alpha sweep (Sec. 6, small and large HBM variants): the
    headline workload on the pinned store with alpha = K / (K + M) of 1 %,
    20 %, 50 % and 80 %; each a build plus the first nb_max batches of 4096
    commands, timed on the launch stream (best of two maps)."""
    d_keys, d_vals, d_ops, d_qk, d_qv, d_out, d_st, bounds = dev_t
    nb = min(nb_max, len(bounds) - 1)
    n_ops = int(bounds[nb])
    out = []
    for apm in alphas:
        p = B.params(wl.cap, wl.vs, alpha_permille=apm)
        sz = B.sizes_of(p)
        best = None
        for _ in range(2):
            m = B.Map(p)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            B.check(m.build(d_keys, d_vals), "bolt_build")
            ev[1].record()
            for bi in range(nb):
                a, b = int(bounds[bi]), int(bounds[bi + 1])
                B.check(m.access(d_ops[a:b], d_qk[a:b], d_qv[a:b], d_out[a:b], d_st[a:b]), "bolt_access_batch")
            B.check(m.flush(), "bolt_flush")
            ev[2].record()
            torch.cuda.synchronize()
            B.check(m.status(), "alpha sweep status")
            m.close()
            r = (ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]))
            best = r if best is None or r[1] < best[1] else best
        out.append({"alpha": apm / 1000, "K": sz["K"], "M": sz["M"], "build_keys_per_s": round(wl.n / (best[0] / 1e3), 1),
                    "ops_per_s": round(n_ops / (best[1] / 1e3), 1),
                    "page_bytes_read_per_op": round(2 * sz["page_bytes"] * sz["M"] / sz["B"], 1)})
        log("alpha %.2f: %s" % (apm / 1000, json.dumps(out[-1])))
    return {"workload": "%s on the pinned store: build, then %d commands in batches of 4096" % (wl.name, n_ops),
            "points": out}


def run_build_heavy(B, torch, synth, autotune):
    """Config 3: build of N=2^26 keys with 8-byte values on the pinned store
    (each build on a fresh map, best of two), its phases from an
    instrumented build (algorithmic GB/s, the sort passes against HBM peak),
    then 2^16 uniform GETs in batches of 4096, every answer checked against
    the build input."""
    t0 = time.time()
    wl = synth.config3()
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(wl.build_keys.view(np.int64)).to(dev)
    vals = torch.from_numpy(wl.build_vals).to(dev)
    log("build-heavy workload %s: n=%d (%.1fs)" % (wl.name, wl.n, time.time() - t0))
    if autotune:
        B.check(B.autotune(1 << 27), "bolt_autotune")  # sort class 2^26, expansion class 2^27
    p = B.params(wl.cap, wl.vs)
    sz = B.sizes_of(p)
    sz["vs"] = wl.vs
    sz["host"] = True
    npad = 1
    while npad < wl.n:
        npad <<= 1
    ms = []
    m = None
    for rep in range(2):
        if m is not None:
            m.close()
        m = B.Map(p)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B.check(m.build(keys, vals), "bolt_build")
        e1.record()
        torch.cuda.synchronize()
        B.check(m.status(), "build status")
        ms.append(e0.elapsed_time(e1))
    # 2^16 uniform GETs, checked against the input
    order = np.argsort(wl.build_keys)
    sk, sv = wl.build_keys[order], wl.build_vals[order]
    got, evs = [], [torch.cuda.Event(enable_timing=True) for _ in range(len(wl.batches) + 1)]
    evs[0].record()
    for bi, (ops, qk, qv) in enumerate(wl.batches):
        q = ops.size
        out = torch.zeros((q, wl.vs), dtype=torch.uint8, device=dev)
        st = torch.zeros(q, dtype=torch.uint8, device=dev)
        B.check(m.access(torch.from_numpy(ops).to(dev), torch.from_numpy(qk.view(np.int64)).to(dev),
                         torch.from_numpy(qv).to(dev), out, st), "bolt_access_batch")
        evs[bi + 1].record()
        got.append((out, st))
    torch.cuda.synchronize()
    B.check(m.status(), "get status")
    n_get = sum(b[0].size for b in wl.batches)
    get_ms = evs[0].elapsed_time(evs[-1])
    for (ops, qk, _), (out, st) in zip(wl.batches, got):
        j = np.searchsorted(sk, qk)
        if not (st.cpu().numpy() == 1).all() or not np.array_equal(out.cpu().numpy(), sv[j]):
            raise SystemExit("build-heavy GET answers differ from the build input")
    m.close()
    # phases of one instrumented build
    pt = B.params(wl.cap, wl.vs)
    pt.flags |= B.BOLT_F_TIMING
    tm = B.Map(pt)
    B.check(tm.build(keys, vals), "bolt_build (timed phases)")
    torch.cuda.synchronize()
    B.check(tm.status(), "timed build status")
    phases = {}
    for cls, (cnt, tot) in sorted(tm.kernel_times().items(), key=lambda kv: -kv[1][1]):
        if cnt == 0 or cls.startswith("acc"):
            continue
        ent = {"launches": cnt, "total_ms": round(tot, 3), "avg_us": round(1e3 * tot / cnt, 2)}
        per, bound = kernel_bytes(cls, sz, wl.n, npad, 0, 0)
        if per is not None:
            gbs = per / (tot / cnt / 1e3) / 1e9
            ent.update({"bytes_per_launch": int(per), "achieved_GBps": round(gbs, 1), "bound": bound,
                        "frac_of_peak": round(gbs / PEAKS[bound], 4)})
        phases[cls] = ent
    tm.close()
    best = min(ms)
    return {"workload": "%s: build of N=2^26 keys with 8-byte values (capacity 2^26), pinned host store; then "
                        "2^16 uniform GETs of present keys in batches of 4096, every answer checked" % wl.name,
            "n": wl.n, "Z": sz["Z"], "page_bytes": sz["page_bytes"], "B": sz["B"], "M": sz["M"],
            "build_ms": round(best, 3), "build_keys_per_s": round(wl.n / (best / 1e3), 1),
            "builds_ms": [round(x, 3) for x in ms],
            "get_ops_per_s": round(n_get / (get_ms / 1e3), 1), "gets_checked": n_get,
            "phases": phases,
            "sort_pass_frac_of_hbm_peak": phases.get("sort_global", {}).get("frac_of_peak")}


def run_multi(B, torch, reps=3):
    """Sixty-four maps (N log-uniform in 2^10..2^22, u64 keys and values),
    each built and then given one GET batch of U[1, 8192] commands (uniform
    present keys, 10 % absent): the many-map calls against 64 one-map calls
    on the same GPU.  Fresh maps for every build repetition (a map is built
    once); map creation is outside the timed regions."""
    import synth

    work = synth.config4()
    dev = torch.device("cuda:0")
    ins = [(torch.from_numpy(w.build_keys.view(np.int64)).to(dev), torch.from_numpy(w.build_vals).to(dev))
           for w in work]
    bts = []
    for w in work:
        ops, keys, _ = w.batches[0]
        q = ops.size
        bts.append((torch.from_numpy(ops).to(dev), torch.from_numpy(keys.view(np.int64)).to(dev),
                    torch.zeros((q, w.vs), dtype=torch.uint8, device=dev),
                    torch.zeros((q, w.vs), dtype=torch.uint8, device=dev),
                    torch.zeros(q, dtype=torch.uint8, device=dev)))
    total_keys = sum(w.n for w in work)
    total_ops = sum(w.batches[0][0].size for w in work)

    def fresh():
        return [B.Map(B.params(w.cap, w.vs)) for w in work]

    tb_many, tb_one, ta_many, ta_one = [], [], [], []
    for r in range(reps):
        ms, ones = fresh(), fresh()
        torch.cuda.synchronize()
        t = time.perf_counter()
        B.check(B.build_many(ms, ins), "bolt_build_many")
        torch.cuda.synchronize()
        tb_many.append(time.perf_counter() - t)
        t = time.perf_counter()
        for m, (k, v) in zip(ones, ins):
            B.check(m.build(k, v), "bolt_build")
        torch.cuda.synchronize()
        tb_one.append(time.perf_counter() - t)
        for _ in range(3):
            # both forms include the write of every rebuilt page (a deferred
            # send is flushed inside the timed region)
            t = time.perf_counter()
            B.check(B.access_many(ms, bts), "bolt_access_many")
            for m in ms:
                B.check(m.flush(), "bolt_flush")
            torch.cuda.synchronize()
            ta_many.append(time.perf_counter() - t)
            t = time.perf_counter()
            for m, b in zip(ones, bts):
                B.check(m.access(*b), "bolt_access_batch")
            for m in ones:
                B.check(m.flush(), "bolt_flush")
            torch.cuda.synchronize()
            ta_one.append(time.perf_counter() - t)
        for m in ms + ones:
            assert m.status() == 0
            m.close()
    med = lambda a: float(np.median(a))
    return {"workload": "64 maps, N log-uniform in [2^10, 2^22], u64 keys/values, one GET batch each of U[1, 8192] "
                        "(10 % absent); observable store in pinned host memory",
            "maps": len(work), "total_keys": total_keys, "total_ops": total_ops,
            "build_keys_per_s": {"many_map": round(total_keys / med(tb_many), 1),
                                 "per_call": round(total_keys / med(tb_one), 1),
                                 "speedup": round(med(tb_one) / med(tb_many), 3)},
            "access_ops_per_s": {"many_map": round(total_ops / med(ta_many), 1),
                                 "per_call": round(total_ops / med(ta_one), 1),
                                 "speedup": round(med(ta_one) / med(ta_many), 3)},
            "ms": {"build_many": round(1e3 * med(tb_many), 3), "build_per_call": round(1e3 * med(tb_one), 3),
                   "access_many": round(1e3 * med(ta_many), 3), "access_per_call": round(1e3 * med(ta_one), 3)}}


def serving_admission(B):
    """How many of config 5's sixteen maps (in open order) the serving budget
    admits at once, with pages in HBM bins and with the decomposed store.
    The budget is the one run_serving uses: the first twelve maps' page
    footprints."""
    import synth

    ns = [n for n, _, _, _ in synth.config5_maps()]

    def fp(n, dec):
        p = B.params(n, 64)
        if dec:
            p.flags |= B.BOLT_F_DECOMPOSED
        return B.server_footprint(p)

    budget = sum(fp(n, False) for n in ns[:12])
    out = {"budget_bytes": budget}
    for dec in (False, True):
        used, k = 0, 0
        for n in ns:
            if used + fp(n, dec) > budget:
                break
            used += fp(n, dec)
            k += 1
        out["decomposed" if dec else "pages"] = {"maps_admitted": k,
                                                  "bytes_all_16": int(sum(fp(n, dec) for n in ns))}
    return out


def run_serving_sealed(B, n_req=4000, seed=0xB0170000 + 56):
    """Sealed commands on the serving path: the sixteen config-5 maps (all
    resident) created with a session key, a backlog of n_req requests
    sealed beforehand by the client helper (a map's k-th request sealed as
    request k), drained as fast as the loop goes; against the same backlog
    in plain commands on plain maps."""
    import ctypes as C

    import synth

    rng = np.random.Generator(np.random.PCG64(seed))
    skey = bytes((5 * i + 1) & 255 for i in range(32))
    specs = synth.config5_maps()
    vs = 64
    reqs = []
    for _ in range(n_req):
        j = int(rng.integers(0, len(specs)))
        q = int(min(4096, max(1, int(2 ** (12 * rng.random())))))
        n, k = specs[j][0], specs[j][1]
        keys = k[rng.integers(0, n, q)]
        ops = np.where(rng.random(q) < 0.1, 1, 0).astype(np.uint8)
        reqs.append((j, ops, keys, rng.integers(0, 256, (q, vs), dtype=np.uint8)))
    out = {"workload": "16 config-5 maps resident; a backlog of %d requests (sizes floor(2^(12u)), 90/10, uniform "
                       "present keys)" % n_req}
    one_ops, one_vals = np.zeros(1, np.uint8), np.zeros((1, vs), np.uint8)
    for mode in ("plain", "sealed"):
        sealed = mode == "sealed"
        srv = B.Server(streams=4)
        ids = [srv.open_map(B.params(n, vs, **({"session_key": skey} if sealed else {})), k, v)
               for n, k, v, _ in specs]
        # one request per map first: every map is resident before the clock starts
        for j in range(len(specs)):
            if sealed:
                srv.submit_sealed(ids[j], B.seal_requests(skey, 1, one_ops, specs[j][1][:1], one_vals, vs), vs)
            else:
                srv.submit(ids[j], one_ops, specs[j][1][:1], one_vals)
        B.check(srv.drain(300000), "drain")
        recs = None
        if sealed:  # the client seals the backlog as requests 2, 3, ... of each map
            seq = [1] * len(specs)
            t = time.perf_counter()
            recs = []
            for j, ops, keys, vals in reqs:
                seq[j] += 1
                recs.append(B.seal_requests(skey, seq[j], ops, keys, vals, vs))
            out["client_seal_s"] = round(time.perf_counter() - t, 2)
        # every request's buffers exist before the clock starts, and the
        # backlog goes in through the C calls directly, so that the loop finds
        # it queued rather than trickling in behind the submissions
        if sealed:
            bufs = [(np.ascontiguousarray(recs[r], dtype=np.uint8), np.zeros((ops.size, 24 + vs), np.uint8))
                    for r, (j, ops, keys, vals) in enumerate(reqs)]
        else:
            bufs = [(np.ascontiguousarray(ops), np.ascontiguousarray(keys, dtype=np.uint64),
                     np.ascontiguousarray(vals), np.zeros((ops.size, vs), np.uint8), np.zeros(ops.size, np.uint8))
                    for j, ops, keys, vals in reqs]
        tk = C.c_uint64()
        srv.reset_stats()
        now = B.bolt_now_ns()
        for r, (j, ops, keys, vals) in enumerate(reqs):
            b = bufs[r]
            if sealed:
                rc = B.bolt_server_submit_sealed(srv.h, ids[j], b[0].ctypes.data, ops.size, b[1].ctypes.data, now,
                                                 C.byref(tk))
            else:
                rc = B.bolt_server_submit(srv.h, ids[j], b[0].ctypes.data, b[1].ctypes.data, b[2].ctypes.data,
                                          b[3].ctypes.data, b[4].ctypes.data, ops.size, now, C.byref(tk))
            if rc != 0:
                raise RuntimeError("submit: %d" % rc)
        B.check(srv.drain(300000), "drain")
        st = srv.stats()
        if st["failed"] or st["completed"] != n_req:
            raise SystemExit("sealed serving: %d of %d requests failed" % (st["failed"], n_req))
        out[mode] = {"req_per_s": round(st["completed"] / st["span_s"], 1),
                     "ops_per_s": round(st["commands"] / st["span_s"], 1),
                     "mean_group_maps": round(st["mean_group_maps"], 2)}
        srv.close()
    out["sealed_relative_to_plain"] = round(out["sealed"]["ops_per_s"] / out["plain"]["ops_per_s"], 4)
    log("serving, sealed commands: %s" % json.dumps(out))
    return out


def run_serving(B, seconds=60.0, rot_seconds=2.0, warm=1.0, pool=1 << 16, seed=0xB0170000 + 55):
    """Sixteen maps (N log-uniform in 2^16..2^24, 64-byte values) behind the
    serving loop.  The HBM budget holds twelve of them at a time: each run
    serves twelve maps for its first half, then closes four and lets four
    waiting ones in, whose builds are admitted as the closed maps leave.  Requests
    arrive as a Poisson process (size floor(2^(12u)) clipped to [1, 4096],
    90 % GET / 10 % PUT, Zipf 0.99 keys over the map's keys, none absent).
    A request's commands are a slice of a per-map pool drawn the same way,
    so the run allocates nothing per request.  First the saturation rate
    (a backlog served as fast as the loop goes), then runs at 0.5x and 0.8x
    of it, each a warm-up, a steady window (twelve resident maps) and a
    rotation window (four maps close, four waiting ones are admitted and
    built while the load goes on; requests to them include their build).
    Latency is arrival to completion."""
    import ctypes as C

    import synth

    rng = np.random.Generator(np.random.PCG64(seed))
    specs = synth.config5_maps()
    vs = 64
    maps = []  # (n, keys, vals)
    for n, k, v, _ in specs:
        maps.append((n, k, v))
    fps = [B.server_footprint(B.params(n, vs)) for n, _, _ in maps]  # what admission counts
    # the budget holds maps 0..11 exactly; at half time of the first run the
    # four largest of them leave for maps 12..15 (smaller together), and the
    # second run swaps them back
    budget = sum(fps[0:12])
    big4 = sorted(range(12), key=lambda j: -fps[j])[:4]
    assert sum(fps[j] for j in range(12, 16)) <= sum(fps[j] for j in big4)
    # command pools: ops 90/10, Zipf(0.99) keys over the map's keys
    pools = []
    for n, k, v in maps:
        ops = np.where(rng.random(pool) < 0.1, 1, 0).astype(np.uint8)
        ranks = synth.zipf_ranks(n, pool, 0.99, rng)
        keys = k[ranks]  # the keys are random, so hot ranks are spread over the key space
        vals = rng.integers(0, 256, (pool, vs), dtype=np.uint8)
        outv = np.zeros((pool, vs), np.uint8)
        outs = np.zeros(pool, np.uint8)
        pools.append((ops, np.ascontiguousarray(keys), vals, outv, outs))
    srv = B.Server(hbm_budget=budget, streams=4)
    t0 = time.perf_counter()
    ids = {}
    for j in range(12):
        ids[j] = srv.open_map(B.params(maps[j][0], vs), maps[j][1], maps[j][2])
    pending = {j: srv.open_map(B.params(maps[j][0], vs), maps[j][1], maps[j][2]) for j in range(12, 16)}  # wait

    def wait_resident(js, limit=120.0):
        t = time.perf_counter()
        while any(srv.map_state(ids[j])[0] != B.BOLT_SRV_RESIDENT for j in js):
            if time.perf_counter() - t > limit:
                raise RuntimeError("maps not admitted: %s" % [srv.map_state(ids[j]) for j in js])
            time.sleep(0.01)

    wait_resident(range(12))
    assert all(srv.map_state(i)[0] == B.BOLT_SRV_WAITING for i in pending.values())
    setup_s = time.perf_counter() - t0
    log("serving: 12 maps resident after %.1fs (budget %.2f GiB, all 16 need %.2f GiB)"
        % (setup_s, budget / 2**30, sum(fps) / 2**30))
    tk = C.c_uint64()
    h = srv.h

    def submit(j, q, arrival_ns):
        ops, keys, vals, outv, outs = pools[j]
        off = int(rng.integers(0, pool - q + 1))
        rc = B.bolt_server_submit(h, ids[j], ops.ctypes.data + off, keys.ctypes.data + 8 * off,
                                  vals.ctypes.data + vs * off, outv.ctypes.data + vs * off, outs.ctypes.data + off,
                                  q, arrival_ns, C.byref(tk))
        if rc != 0:
            raise RuntimeError("submit: %d" % rc)
        return q

    def req_size():
        return int(min(4096, max(1, int(2 ** (12 * rng.random())))))

    # saturation: a backlog over the twelve resident maps
    srv.reset_stats()
    now = B.bolt_now_ns()
    live = sorted(ids)
    for _ in range(6000):
        submit(live[int(rng.integers(0, len(live)))], req_size(), now)
    B.check(srv.drain(300000), "drain")
    sat = srv.stats()
    sat_rps = sat["completed"] / sat["span_s"]
    sat_ops = sat["commands"] / sat["span_s"]
    log("serving saturation: %.0f req/s, %.3g ops/s" % (sat_rps, sat_ops))
    out = {"workload": "16 maps, N log-uniform in [2^16, 2^24], 64-byte values; Poisson request batches of "
                       "floor(2^(12u)) in [1, 4096] commands, 90 % GET / 10 % PUT, Zipf 0.99, none absent; "
                       "12 maps resident under the HBM budget, 4 rotated per run",
           "hbm_budget_bytes": budget, "all_maps_bytes": int(sum(fps)), "setup_s": round(setup_s, 2),
           "saturation": {"req_per_s": round(sat_rps, 1), "ops_per_s": round(sat_ops, 1),
                          "lat_p50_ms": round(sat["lat_p50_ms"], 3), "lat_p99_ms": round(sat["lat_p99_ms"], 3),
                          "mean_group_maps": round(sat["mean_group_maps"], 2),
                          "mean_group_commands": round(sat["mean_group_commands"], 1)},
           "runs": []}
    # open-loop runs; each rotates four maps at half time
    rot = [(big4, list(range(12, 16))), (list(range(12, 16)), big4)]
    for run, frac in enumerate((0.5, 0.8)):
        rate = frac * sat_rps
        closing, opening = rot[run]
        if run:  # the maps to admit mid-run are opened (and wait) before the run
            pending = {j: srv.open_map(B.params(maps[j][0], vs), maps[j][1], maps[j][2]) for j in opening}
        assert all(srv.map_state(pending[j])[0] == B.BOLT_SRV_WAITING for j in opening)
        srv.reset_stats()
        start = B.bolt_now_ns()
        t_warm = start + int(warm * 1e9)
        t_rot = t_warm + int(seconds * 1e9)
        t_end = t_rot + int(rot_seconds * 1e9)
        t = start
        phase = 0  # 0 warm-up, 1 steady, 2 rotation
        steady = None

        def summary(st, secs):
            span = max(st["span_s"], 1e-9)
            return {"seconds": secs, "requests": st["completed"], "failed": st["failed"],
                    "completed_req_per_s": round(st["completed"] / span, 1),
                    "ops_per_s": round(st["commands"] / span, 1),
                    "lat_p50_ms": round(st["lat_p50_ms"], 3), "lat_p99_ms": round(st["lat_p99_ms"], 3),
                    "lat_max_ms": round(st["lat_max_ms"], 3), "queue_peak": st["queue_peak"],
                    "mean_group_maps": round(st["mean_group_maps"], 2),
                    "mean_group_commands": round(st["mean_group_commands"], 1),
                    "maps_admitted": st["maps_admitted"], "hbm_peak_bytes": st["hbm_peak"]}

        next_note = start + int(10e9)
        while True:
            t += int(rng.exponential(1.0 / rate) * 1e9)
            if t >= t_end:
                break
            if t >= next_note:  # a progress line every ten seconds of the run
                log("serving at %.1fx: %.0f s of %.0f s" % (frac, (t - start) / 1e9, (t_end - start) / 1e9))
                next_note += int(10e9)
            if phase == 0 and t >= t_warm:
                while B.bolt_now_ns() < t_warm:
                    pass
                srv.reset_stats()
                phase = 1
            if phase == 1 and t >= t_rot:
                while B.bolt_now_ns() < t_rot:
                    pass
                steady = summary(srv.stats(), seconds)
                srv.reset_stats()
                for j in closing:
                    B.check(srv.close_map(ids.pop(j)), "close_map")
                for j in opening:
                    ids[j] = pending[j]
                live = sorted(ids)
                phase = 2
            while B.bolt_now_ns() < t:
                pass
            submit(live[int(rng.integers(0, len(live)))], req_size(), t)
        B.check(srv.drain(300000), "drain")
        rotation = summary(srv.stats(), rot_seconds)
        lag = (B.bolt_now_ns() - t_end) / 1e9
        out["runs"].append({"load": frac, "offered_req_per_s": round(rate, 1), "steady": steady,
                            "rotation": rotation, "drain_s": round(lag, 3), "warmup_s": warm})
        log("serving at %.1fx: %s" % (frac, json.dumps(out["runs"][-1])))
    srv.close()
    return out


def run_dynamics(B, torch, accesses, log2n=20, batch=4096, seed=0xB0170000 + 61):
    """The paper's validation of the bin, HBM and stash bounds (Sec. 4.3,
    "Dimensions in practice"), on the GPU with the batched path: N = 2^log2n
    keys, `accesses` uniform random GETs over them in batches of `batch`,
    for c in {8, 16} and alpha in {0.01, 0.2, 0.5}, device observable store,
    BOLT_F_WATCH tracking the largest bin load and the HBM-bin items at
    every batch end.  The bounds are Claim 4.2 (l_max = Z), Claim 4.3
    (K c + l_max sqrt(K ln N)) and Claim 4.4 ((1 + alpha) M / 2 +
    l_max sqrt(M ln N)), O() constants 1.  The query stream cycles through
    a pool of 2048 random batches drawn once per configuration."""
    import math

    import synth

    n = 1 << log2n
    dev = torch.device("cuda:0")
    keys = synth.keys(n, seed)
    vals = synth.values(n, 8, seed + 1)
    dk = torch.from_numpy(keys.view(np.int64)).to(dev)
    dv = torch.from_numpy(vals).to(dev)
    g = torch.Generator(device=dev)
    pool = 2048
    out = {"workload": "N=2^%d keys, %d uniform random GETs in batches of %d, device observable store" % (
        log2n, accesses, batch), "configs": []}
    ops = torch.zeros(batch, dtype=torch.uint8, device=dev)
    vin = torch.zeros((batch, 8), dtype=torch.uint8, device=dev)
    vout = torch.zeros((batch, 8), dtype=torch.uint8, device=dev)
    st = torch.zeros(batch, dtype=torch.uint8, device=dev)
    nb = accesses // batch
    for c in (8, 16):
        for alpha_pm in (10, 200, 500):
            g.manual_seed(seed + 1000 * c + alpha_pm)
            qk = dk[torch.randint(0, n, (pool, batch), device=dev, generator=g)]
            p = B.params(n, 8, c=c, alpha_permille=alpha_pm, observable=B.BOLT_OBS_DEVICE)
            p.flags |= B.BOLT_F_WATCH
            m = B.Map(p)
            B.check(m.build(dk, dv), "bolt_build")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            overflow_at = None
            done = 0
            for b in range(nb):
                B.check(m.access(ops, qk[b % pool], vin, vout, st), "bolt_access_batch")
                done += 1
                if b % 4096 == 4095 or b == nb - 1:
                    rc = m.status()  # synchronises; a capacity error poisons the map
                    if rc != 0:
                        overflow_at = {"error": B._NAMES.get(rc, rc), "within_accesses": done * batch}
                        break
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            sz = m.sizes
            s_ = m.stats()  # a poisoned map still reports its counters and watch marks
            K, M, Z = sz["K"], sz["M"], sz["lmax"]  # the bounds use l_max (the pages hold Z >= l_max)
            a = alpha_pm / 1000.0
            b43 = K * c + Z * math.sqrt(K * math.log(n))
            b44 = (1 + a) * M / 2 + Z * math.sqrt(M * math.log(n))
            ent = {"c": c, "alpha": a, "accesses": done * batch, "seconds": round(secs, 2),
                   "ops_per_s": round(done * batch / secs, 1), "K": K, "M": M, "overflow": overflow_at,
                   "bin_load": {"max": s_["load_highwater"], "bound": Z, "slack": Z - s_["load_highwater"],
                                "rel_slack": round((Z - s_["load_highwater"]) / Z, 4)},
                   "hbm_load": {"max": s_["hbm_load_highwater"], "bound": round(b43, 1),
                                "slack": round(b43 - s_["hbm_load_highwater"], 1),
                                "rel_slack": round((b43 - s_["hbm_load_highwater"]) / b43, 4)},
                   "stash": {"max": s_["stash_highwater"], "bound": round(b44, 1),
                             "slack": round(b44 - s_["stash_highwater"], 1),
                             "rel_slack": round((b44 - s_["stash_highwater"]) / b44, 4),
                             "max_fraction_of_N": round(s_["stash_highwater"] / n, 4)},
                   "max_row": s_["max_row"], "row_slots": p.pm_row_slots}
            out["configs"].append(ent)
            log("dynamics c=%d alpha=%.2f: %s" % (c, a, json.dumps(ent)))
            m.close()
            del qk
    return out


def host_cpu():
    """The host's core count (all of them and those this process may use)
    and CPU model, from the kernel's own tables."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cores": usable, "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(n_batches, full_batches=64):
    """CPU baselines on the GPU machine's host cores, as they stand:
    * the oracle (O2, scalar C, one thread) on a bounded sample: the same
      workload scaled to N=2^20 (64-byte values, Zipf 0.99, 5 % absent,
      90/10), its build plus n_batches batches of 4096 (the headline
      baseline);
    * the same oracle built with OpenMP over all usable cores, on the real
      config-2 size (N=2^24 + 2^16 capacity): build plus full_batches
      batches of 4096;
    * the plain definition O1 (a C hash table, one thread) on the same
      full-size workload."""
    import oracle as O
    import synth

    host = host_cpu()
    n = 1 << 20
    wl = synth.config2(n=n, n_ops=n_batches * 4096, batch=4096, headroom=1 << 16)
    m = O.OracleMap(wl.cap, wl.vs, key=bytes(range(32)))
    t = time.perf_counter()
    assert m.build(wl.build_keys, wl.build_vals) == 0
    tb = time.perf_counter() - t
    t = time.perf_counter()
    for ops, ks, vs_ in wl.batches:
        rc, _, _ = m.access(ops, ks, vs_)
        assert rc == 0
    tq = time.perf_counter() - t
    m.close()
    del wl
    log("cpu baseline: oracle, one thread, N=2^20: build %.1fs, %d batches %.1fs" % (tb, n_batches, tq))

    full = synth.config2(n_batches=full_batches)
    om = O.OracleMap(full.cap, full.vs, key=bytes(range(32)), lib=O.load_openmp())
    t = time.perf_counter()
    assert om.build(full.build_keys, full.build_vals) == 0
    otb = time.perf_counter() - t
    t = time.perf_counter()
    for ops, ks, vs_ in full.batches:
        assert om.access(ops, ks, vs_)[0] == 0
    otq = time.perf_counter() - t
    om.close()
    log("cpu baseline: oracle with OpenMP, N=2^24: build %.1fs, %d batches %.1fs" % (otb, full_batches, otq))

    pc = O.PlainMapC(full.cap, full.vs)
    t = time.perf_counter()
    assert pc.build(full.build_keys, full.build_vals) == 0
    ptb = time.perf_counter() - t
    t = time.perf_counter()
    for ops, ks, vs_ in full.batches:
        assert pc.access(ops, ks, vs_)[0] == 0
    ptq = time.perf_counter() - t
    pc.close()
    n_full = full.n_ops
    return {"value": round(n_batches * 4096 / tq, 1), "unit": "ops/s", "cores": 1, "kind": "oracle",
            "build_keys_per_s": round(n / tb, 1),
            "sample": "oracle (scalar C, one thread) on the same workload scaled to N=2^20: build of 2^20 keys "
                      "(%.1fs) then %d batches of 4096 commands (%.1fs)" % (tb, n_batches, tq),
            "host": host,
            "openmp": {"ops_per_s": round(n_full / otq, 1), "build_keys_per_s": round(full.n / otb, 1),
                       "cores": host["usable_cores"] if not host["omp_num_threads"] else
                       min(host["usable_cores"], int(host["omp_num_threads"])),
                       "kind": "oracle built with OpenMP",
                       "sample": "config 2 at full size: build of 2^24 keys (%.1fs) then %d batches of 4096 "
                                 "commands (%.1fs)" % (otb, full_batches, otq)},
            "plain_o1": {"ops_per_s": round(n_full / ptq, 1), "build_keys_per_s": round(full.n / ptb, 1),
                         "cores": 1, "kind": "plain definition (C hash table, not oblivious)",
                         "sample": "config 2 at full size: 2^24 inserts (%.2fs) then %d batches of 4096 "
                                   "commands (%.2fs)" % (ptb, full_batches, ptq)}}


if __name__ == "__main__":
    main()
