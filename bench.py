#!/usr/bin/env python3
"""Benchmark of sgn(gamma5 Dw(mu)) x on one MI355X.

Workload: 16^4 lattice, mu = 0.3 (two-sided Lanczos), m_w = -1, link width
eps = 0.8 (gauge seed 0), one complex Gaussian source (seed 0), FP64.  One
step is one whole application of the nested method (outer basis, nested
small problem with Roberts-Higham, lift) at the (k, l) that reach relative
accuracy 1e-8; the plain non-nested method is timed beside it at the same k.
Accuracy of both is measured live against a non-nested reference run at
k + 500.  Inputs are resident in device memory before timing starts.

The JSON line also carries the roofline of the dominant kernel (the fused
two-sided Lanczos stencil step), its average duration measured with HIP
events on the launch stream over the timed steps, and the CPU oracle timed
on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (16, 16, 16, 16)
MU = 0.3
M_W = -1.0
EPS = 0.8
# algorithmic bytes per site of the fused two-sided Lanczos stencil step in
# FP64: 4 links (576 B) + v_j, w_j, v_{j-1}, w_{j-1} read (4 x 192 B) + p, q
# written (2 x 192 B)
K1_BYTES_PER_SITE = 576 + 4 * 192 + 2 * 192
# every PROFILE_EVERY-th outer step of each timed application has its two
# kernels bracketed by HIP events bound to the launches (a sample: events on
# every launch would slow the timed run itself by about 15%, on every tenth
# step by about 0.7%)
PROFILE_EVERY = 25
HBM_PEAK_GBS = 8000.0
PROFILE_PMC = os.path.join(ROOT, "profiles", "k_bil1_16x16x16x16_pmc.json")


def step_kernel_bytes(hermitian: bool, prec: int) -> tuple:
    """Algorithmic bytes per site of the two kernels of one outer step: links
    read once, every vector read or written once (FP64 / FP32 spinors of 12
    complex entries; FP64, FP32 or BF16 two-row links)."""
    spinor = 12 * (16 if prec == 0 else 8)
    links = {0: 4 * 9 * 16, 1: 4 * 9 * 8, 2: 4 * 6 * 4}[prec]
    if hermitian:  # K1: v_j, v_{j-1} in, p out; K2: p, v_j in, v_{j+1} out
        return links + 3 * spinor, 3 * spinor
    # K1: v_j, w_j, v_{j-1}, w_{j-1} in, p, q out; K2: p, q, v_j, w_j in, v_{j+1}, w_{j+1} out
    return links + 6 * spinor, 6 * spinor


def copy_rate(torch, dev) -> float:
    """GB/s of a plain device copy of 1 GiB (read 1 GiB, write 1 GiB): larger
    than the Infinity Cache, so it shows what streaming from HBM reaches."""
    n = 1024 * 1024 * 1024 // 16
    src = torch.ones(n, dtype=torch.complex128, device=dev)
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(4):
        ev[0].record()
        torch.mul(src, 2.0, out=dst)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    del src, dst
    return 2 * n * 16 / (best / 1e3) / 1e9


def stream_ceiling(torch, nk, dev, nbytes=1024 ** 3):
    """What this library's own streaming kernels reach (nk_stream_device):
    read-only, copy and triad over arrays of nbytes each (1 GiB, four times
    the Infinity Cache, so every pass streams from HBM), 16 bytes per lane,
    the best over a sweep of grid sizes, timed with HIP events on the launch
    stream.  Bytes: read-only n, copy 2 n, triad 3 n."""
    n = nbytes // 16
    a = torch.ones(n, dtype=torch.complex128, device=dev)
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {"bytes_per_array": nbytes}
    for kind, name, mult in ((0, "read_only", 1), (1, "copy", 2), (2, "triad", 3)):
        best = (float("inf"), 0)
        for blocks in (1024, 2048, 4096, 8192, 16384):
            nk.nk_stream_device(kind, a, b if kind == 2 else None, c, blocks)
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(5):
                nk.nk_stream_device(kind, a, b if kind == 2 else None, c, blocks)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / 5
            if ms < best[0]:
                best = (ms, blocks)
        gbs = mult * nbytes / (best[0] / 1e3) / 1e9
        out[name] = {"GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "ms": best[0], "blocks": best[1]}
    del a, b, c
    return out


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("krylov.hip", "stencil.h", "nk_internal.h", "layout.hip"):
        with open(os.path.join(ROOT, "paper_0910_2918_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stencil_rates(torch, nk, latgen, dev, copy_gbs, reps=100, nsets=10):
    """The stand-alone stencil at 16^4, mu = 0.3, FP64, on vectors in the
    library's packed layout (one kernel launch per application): the single
    operator gamma5 Dw (960 algorithmic B/site: 4 links, one vector in, one
    out) and the fused pair (A v, A^dag w; 1344 B/site).  'warm' repeats the
    application on one (gauge, in, out) set, which stays resident in the 256 MB
    Infinity Cache; 'cold' cycles nsets distinct sets (their gauge fields hold
    the same values in separate buffers), 629 MB for the single operator and
    880 MB for the pair, more than twice that cache.  reps back-to-back
    launches between two HIP events on the launch stream (the ctypes calls are
    bound beforehand so that the host keeps ahead of the device)."""
    import ctypes as C

    import numpy as np

    V = DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3]
    u = latgen.random_gauge(DIMS, EPS, 0)
    src = latgen.random_sources(DIMS, 2, 9)
    lib = nk.library()
    sets = []
    for i in range(nsets):
        lat = nk.Lattice(DIMS)
        nk.nk_gauge_set(lat.h, u)
        canon = [torch.from_numpy(np.ascontiguousarray(src[r]).reshape(-1)).to(dev) for r in range(2)]
        vp, wp = torch.empty_like(canon[0]), torch.empty_like(canon[0])
        nk.nk_spinor_pack_device(lat.h, canon[0], vp)
        nk.nk_spinor_pack_device(lat.h, canon[1], wp)
        sets.append((lat, vp, wp, torch.empty_like(vp), torch.empty_like(vp)))
        del canon
    torch.cuda.synchronize()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    vptr = lambda t: C.c_void_p(t.data_ptr())
    single = [(lib.nk_apply_dw_packed_device, (st[0].h, M_W, MU, 1, vptr(st[1]), vptr(st[3]), stream))
              for st in sets]
    pair = [(lib.nk_apply_pair_packed_device, (st[0].h, M_W, MU, vptr(st[1]), vptr(st[2]), vptr(st[3]),
                                               vptr(st[4]), stream)) for st in sets]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def run(calls):
        for f, a in calls[:4]:  # warm-up
            if f(*a):
                raise nk.NKError(-1, nk.nk_last_error())
        seq = [calls[i % len(calls)] for i in range(reps)]
        torch.cuda.synchronize()
        ev[0].record()
        for f, a in seq:
            f(*a)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) * 1e3 / reps

    out = {"lattice": "16^4", "mu": MU, "launches": reps, "cold_sets": nsets}
    for name, calls, bps in (("single", single, 960), ("pair", pair, 1344)):
        for temp, cl in (("warm", calls[:1]), ("cold", calls)):
            us = run(cl)
            gbs = bps * V / us / 1e3
            out[f"{name}_{temp}"] = {"us": us, "bytes_per_site": bps, "GBps": gbs,
                                     "frac_of_peak": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs}
    for st in sets:
        st[0].close()
    del sets, single, pair
    return out


def rel(a, b) -> float:
    import torch

    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def host_cpu():
    """nproc (the CPUs this process may run on) and the CPU model from lscpu."""
    import subprocess

    try:
        nproc = len(os.sched_getaffinity(0))
    except Exception:
        nproc = os.cpu_count() or 1
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return nproc, model


HK16 = os.path.join(ROOT, "tests", "golden", "hk_16x16x16x16_mu0.3_eps0.8_k500.npz")


def cpu_baseline(k: int, ell: int, sample_steps: int):
    """The CPU oracle on a bounded sample of the workload, scaled to applies/s."""
    import numpy as np

    import latgen
    from oracle import krylov as K
    from oracle import nested as N
    from oracle import wilson as W

    try:
        from threadpoolctl import threadpool_info

        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        blas_threads = 1
    nproc, model = host_cpu()
    u = latgen.random_gauge(DIMS, EPS, 0)
    x = latgen.random_sources(DIMS, 1, 0)[0]
    f = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, MU).reshape(-1)
    fd = lambda v: W.a_apply(u, v.reshape(x.shape), M_W, -MU).reshape(-1)
    t0 = time.perf_counter()
    kr = K.two_sided_lanczos(f, fd, x.reshape(-1), sample_steps)
    t_step = (time.perf_counter() - t0) / sample_steps
    # lift: the same dense product over the sample's columns, scaled to k columns
    z = np.ones(sample_steps, np.complex128)
    t0 = time.perf_counter()
    _ = kr.V @ z
    t_lift = (time.perf_counter() - t0) * k / sample_steps
    # the small problem at full size on this workload's own Ritz matrix H_k
    # (written by the oracle, tests/golden/make_hk.py); without that file, on
    # the Ritz matrix of the same order from a 4^4 lattice
    if os.path.exists(HK16) and k <= 500:
        d = np.load(HK16)
        H = K.Tridiag(d["alpha"][:k], d["beta"][: k - 1], d["delta"][: k - 1])
        hk_src = "this workload's H_k (16^4, written by the oracle)"
    else:
        dims_s = (4, 4, 4, 4)
        us = latgen.random_gauge(dims_s, EPS, 0)
        xs = latgen.random_sources(dims_s, 1, 0)[0]
        fs = lambda v: W.a_apply(us, v.reshape(xs.shape), M_W, MU).reshape(-1)
        fds = lambda v: W.a_apply(us, v.reshape(xs.shape), M_W, -MU).reshape(-1)
        H = K.two_sided_lanczos(fs, fds, xs.reshape(-1), k).H
        hk_src = "the H_k of the same order from a 4^4 lattice"
    t0 = time.perf_counter()
    N.small_sign(H, ell, False)
    t_small = time.perf_counter() - t0
    t0 = time.perf_counter()
    N.small_sign(H, 0, False)
    t_small_plain = time.perf_counter() - t0
    t_apply = k * t_step + t_small + t_lift
    return {
        "value": 1.0 / t_apply,
        "unit": "applies/s",
        "cores": int(blas_threads),
        "kind": "oracle",
        "sample": (f"{sample_steps} two-sided Lanczos steps of the oracle at 16^4 (numpy, single-threaded stencil) "
                   f"scaled to k={k}, plus the oracle's full nested small problem (k={k}, l={ell}; LAPACK with "
                   f"{blas_threads} BLAS threads) on {hk_src}, and the lift product scaled from {sample_steps} "
                   f"columns"),
        "nproc": nproc,
        "cpu_model": model,
        "threads": {"stencil": 1, "small_problem_and_lift": int(blas_threads)},
        "t_step_s": t_step,
        "t_small_s": t_small,
        "t_small_plain_s": t_small_plain,
        "t_lift_s": t_lift,
        "plain_applies_per_s": 1.0 / (k * t_step + t_small_plain + t_lift),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=500)
    ap.add_argument("--ell", type=int, default=60)
    ap.add_argument("--kref-extra", type=int, default=500)
    ap.add_argument("--cpu-sample-steps", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8, help="sources of the lockstep run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--target", type=float, default=1e-8)
    ap.add_argument("--probe", action="store_true",
                    help="short run for hardware counters: a copy kernel of known size (1 GiB read, 1 GiB "
                         "written, larger than the 256 MB Infinity Cache) three times, then one application "
                         "at k=20, l=5 of the same workload (same stencil dispatches as the timed run), one "
                         "deflated application and four sources in lockstep at the same k, l, then the "
                         "stand-alone stencil (single operator and fused pair, warm and cold, 20 launches each)")
    ap.add_argument("--calibrate", action="store_true",
                    help="print the relative error of plain and nested runs over a grid of (k, l)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the library has no multi-GPU path",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import latgen
    from paper_0910_2918_amd import nk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    lib = nk.library()  # fails loudly if libnk.so is missing
    del lib
    dev = torch.device("cuda:0")
    lat = nk.Lattice(DIMS)
    nk.nk_gauge_set(lat.h, latgen.random_gauge(DIMS, EPS, 0))
    x = torch.from_numpy(latgen.random_sources(DIMS, 1, 0)[0].reshape(-1)).to(dev)
    y = torch.empty_like(x)
    yref = torch.empty_like(x)

    def params(k, ell, profile=0, scaling=0, nrhs=1, block=0):
        return nk.nk_sign_params_default(k=k, ell=ell, mu=MU, m_w=M_W, profile=profile, rh_scaling=scaling,
                                         nrhs=nrhs, block=block)

    # the learned Roberts-Higham scaling (trained weights shipped with the package)
    from paper_0910_2918_amd import rh_train

    have_model = os.path.exists(rh_train.WEIGHTS)
    if have_model:
        nk.nk_rh_model_set(np.load(rh_train.WEIGHTS).astype(np.float32))
    LEARNED = nk.NK_RH_LEARNED if have_model else nk.NK_RH_NONE

    if args.probe:
        n = 1024 * 1024 * 1024 // 16
        src = torch.ones(n, dtype=torch.complex128, device=dev)
        dst = torch.empty_like(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        times = []
        for _ in range(3):
            ev[0].record()
            torch.mul(src, 2.0, out=dst)
            ev[1].record()
            torch.cuda.synchronize()
            times.append(ev[0].elapsed_time(ev[1]))
        nk.nk_sign_apply_device(lat.h, params(20, 5), x, y)
        # one deflated application (m = 32 seeded unit vectors standing in for
        # eigenpairs) for the deflation kernels' counters
        md = 32
        dv = [latgen.random_sources(DIMS, md, sd).reshape(md, -1) for sd in (6, 7)]
        rd, ld = (torch.from_numpy(a / np.linalg.norm(a, axis=1, keepdims=True)).to(dev).reshape(-1) for a in dv)
        lamd = np.array([1.0 if i % 2 == 0 else -1.0 for i in range(md)], dtype=np.complex128)
        nk.nk_sign_apply_deflated_device(lat.h, params(20, 5), lamd, rd, ld, x, y)
        # four sources in lockstep (block = 1) at k = 20, l = 5: the lockstep
        # stencil's counters (k_blk1, one source per workgroup as tuned)
        xb4 = torch.from_numpy(latgen.random_sources(DIMS, 4, 1).reshape(-1)).to(dev)
        yb4 = torch.empty_like(xb4)
        nk.nk_sign_apply_device(lat.h, params(20, 5, nrhs=4, block=1), xb4, yb4)
        torch.cuda.synchronize()
        gbs = 2 * n * 16 / (min(times) / 1e3) / 1e9
        del src, dst, xb4, yb4, rd, ld
        # the stand-alone stencil, warm and cold, 20 launches each (the only
        # dispatches of k_apply in the probe, in the order single warm, single
        # cold, pair warm, pair cold, each after its warm-up launches)
        st = stencil_rates(torch, nk, latgen, dev, gbs, reps=20)
        print(json.dumps({"probe": "done", "copy_bytes_read": n * 16, "copy_bytes_written": n * 16,
                          "copy_ms": times, "copy_GBps": gbs,
                          "stencil_us": {k: v["us"] for k, v in st.items() if isinstance(v, dict)}}))
        lat.close()
        return 0

    if args.calibrate:
        kref = 1400
        nk.nk_sign_apply_device(lat.h, params(kref, 0), x, yref)
        for k in range(350, 651, 25):
            nk.nk_sign_apply_device(lat.h, params(k, 0), x, y)
            row = {"k": k, "plain": rel(y, yref)}
            for ell in (k // 10, k // 8, k // 6, k // 5, k // 4):
                nk.nk_sign_apply_device(lat.h, params(k, ell), x, y)
                row[f"l={ell}"] = rel(y, yref)
            print(json.dumps(row), flush=True)
        lat.close()
        return 0

    # accuracy, untimed: reference = non-nested at k + kref_extra
    kref = args.k + args.kref_extra
    nk.nk_sign_apply_device(lat.h, params(kref, 0), x, yref)
    nk.nk_sign_apply_device(lat.h, params(args.k, args.ell, scaling=LEARNED), x, y)
    eps_nested = rel(y, yref)
    nk.nk_sign_apply_device(lat.h, params(args.k, 0), x, y)
    eps_plain = rel(y, yref)

    def timed(nsteps, **kw):
        """Wall time per application over nsteps after one warm-up, with the same
        kernel-event sampling as the headline's timed steps; summed info fields."""
        kw.setdefault("profile", PROFILE_EVERY)
        nk.nk_sign_apply_device(lat.h, params(**kw), x, y)
        torch.cuda.synchronize()
        acc = {"t_stencil_ms": 0.0, "n_stencil": 0, "t_update_ms": 0.0, "n_update": 0, "t_basis_ms": 0.0,
               "t_small_ms": 0.0, "t_lift_ms": 0.0, "rh_iters": 0}
        t0 = time.perf_counter()
        for _ in range(nsteps):
            info, rc = nk.nk_sign_apply_device(lat.h, params(**kw), x, y)
            for f in acc:
                acc[f] = acc[f] + getattr(info, f) if f != "rh_iters" else info.rh_iters
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / nsteps, acc

    # the headline form: nested with learned scaling; warmup, then K timed steps
    # (kernel durations sampled with HIP events bound to the launches)
    for _ in range(args.warmup):
        nk.nk_sign_apply_device(lat.h, params(args.k, args.ell, scaling=LEARNED), x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = {"t_stencil_ms": 0.0, "n_stencil": 0, "t_update_ms": 0.0, "n_update": 0}
    ph = {"basis": 0.0, "small": 0.0, "lift": 0.0}
    rh_iters = 0
    for _ in range(args.steps):
        info, rc = nk.nk_sign_apply_device(lat.h, params(args.k, args.ell, profile=PROFILE_EVERY, scaling=LEARNED),
                                           x, y)
        for f in st:
            st[f] += getattr(info, f)
        ph["basis"] += info.t_basis_ms
        ph["small"] += info.t_small_ms
        ph["lift"] += info.t_lift_ms
        rh_iters = info.rh_iters
    torch.cuda.synchronize()
    t_nested = (time.perf_counter() - t0) / args.steps
    t_st, n_st, t_up, n_up = st["t_stencil_ms"], st["n_stencil"], st["t_update_ms"], st["n_update"]

    # the other forms at the same k, as many steps and the same event sampling
    # as the headline (timed for the comparison only)
    nside = max(1, args.steps // 2)
    t_plain, info_p = timed(args.steps, k=args.k, ell=0)
    t_nested_u, info_u = timed(args.steps, k=args.k, ell=args.ell)
    t_nested_d, info_d = timed(args.steps, k=args.k, ell=args.ell, scaling=nk.NK_RH_DET)
    # the three nested scalings and the plain form interleaved, one application of
    # each per round with the order rotated every round, so that clock drift
    # between timing blocks cancels; every timed application follows the same
    # untimed one (the headline form), so that no form inherits the state
    # another leaves behind (the plain form's long, latency-bound small problem
    # would otherwise slow whichever form comes next): median wall time of
    # each form's applications (each bracketed by synchronisation)
    inter_forms = {"nested_learned": dict(scaling=LEARNED), "nested_determinant": dict(scaling=nk.NK_RH_DET),
                   "nested_unscaled": dict(scaling=nk.NK_RH_NONE), "plain_unscaled": dict(ell=0)}
    inter_t = {f: [] for f in inter_forms}
    names = list(inter_forms)
    nrounds = 4 * max(2, (args.steps + 3) // 4)
    p_lead = params(args.k, args.ell, profile=PROFILE_EVERY, scaling=LEARNED)
    for rr in range(nrounds):
        for f in names[rr % 4:] + names[:rr % 4]:
            kw = inter_forms[f]
            kw2 = dict(k=args.k, ell=args.ell, profile=PROFILE_EVERY)
            kw2.update(kw)
            nk.nk_sign_apply_device(lat.h, p_lead, x, y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nk.nk_sign_apply_device(lat.h, params(**kw2), x, y)
            torch.cuda.synchronize()
            inter_t[f].append(time.perf_counter() - t0)
    forms_interleaved = {f: {"applies_per_s": 1.0 / float(np.median(v)), "ms_median": float(np.median(v)) * 1e3,
                             "ms_min": min(v) * 1e3, "rounds": len(v)} for f, v in inter_t.items()}
    # many sources in lockstep (nested, learned scaling): per-source rate
    nb = args.batch
    xb = torch.from_numpy(latgen.random_sources(DIMS, nb, 1).reshape(-1)).to(dev)
    yb = torch.empty_like(xb)
    pb = params(args.k, args.ell, scaling=LEARNED, nrhs=nb, block=2)
    nk.nk_sign_apply_device(lat.h, pb, xb, yb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nside):
        info_b, _ = nk.nk_sign_apply_device(lat.h, pb, xb, yb)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / nside
    del xb, yb

    # deflation (Sec. 2) on this lattice at mu = 0.3 with its own critical
    # eigenpairs: the 16 eigenvalues of gamma5 Dw(0.3) nearest the imaginary
    # axis with right and left vectors from the library's two-sided
    # eigensolver (block of 32, degree 40), then the deflated nested sign at
    # the same (k, l) and scaling (its time, its error against the reference
    # beside the undeflated one), the smallest k on a grid of 50 at which the
    # deflated nested sign reaches the target, and the deflation's own cost
    # (the median difference between deflated and undeflated applications at
    # k = 4, where the Krylov part, the same in both, is short)
    md, pblk, deg_c = 16, 32, 40
    nvec_c = 12 * DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3]
    V0c = torch.from_numpy(latgen.random_sources(DIMS, pblk, 11).reshape(-1)).to(dev)
    rd = torch.empty(md * nvec_c, dtype=torch.complex128, device=dev)
    ld = torch.empty_like(rd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lamd, passes_c, res_c, rc_c = nk.nk_eig_critical_device(lat.h, M_W, MU, md, pblk, deg_c, 1e-10, 100, V0c, rd,
                                                           ld)
    t_eig_c = time.perf_counter() - t0
    del V0c
    pd = params(args.k, args.ell, scaling=LEARNED)
    nk.nk_sign_apply_deflated_device(lat.h, pd, lamd, rd, ld, x, y)
    torch.cuda.synchronize()
    e_defl = rel(y, yref)
    t0 = time.perf_counter()
    for _ in range(nside):
        nk.nk_sign_apply_deflated_device(lat.h, pd, lamd, rd, ld, x, y)
    torch.cuda.synchronize()
    t_d = (time.perf_counter() - t0) / nside
    k_defl = None
    for kk in range(300, args.k + 1, 50):
        nk.nk_sign_apply_deflated_device(lat.h, params(kk, args.ell, scaling=LEARNED), lamd, rd, ld, x, y)
        if rel(y, yref) <= args.target:
            k_defl = kk
            break
    # the deflated form at the smallest k that meets the target (same l):
    # what deflation buys once the eigenpairs exist
    t_dk = None
    if k_defl is not None:
        pk = params(k_defl, args.ell, scaling=LEARNED)
        nk.nk_sign_apply_deflated_device(lat.h, pk, lamd, rd, ld, x, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nside):
            nk.nk_sign_apply_deflated_device(lat.h, pk, lamd, rd, ld, x, y)
        torch.cuda.synchronize()
        t_dk = (time.perf_counter() - t0) / nside
    p4 = params(4, 0)
    diffs = []
    for _ in range(21):
        t0 = time.perf_counter()
        nk.nk_sign_apply_deflated_device(lat.h, p4, lamd, rd, ld, x, y)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nk.nk_sign_apply_device(lat.h, p4, x, y)
        torch.cuda.synchronize()
        diffs.append((t1 - t0) - (time.perf_counter() - t1))
    t_over = float(np.median(diffs[1:]))
    nvec = nvec_c * 16
    # L^dag x, the projected source and its norm, the exact part: 3 m + 6 vectors
    defl_bytes = (3 * md + 6) * nvec
    deflation = {"m": md, "k": args.k, "ell": args.ell, "mu": MU,
                 "eigensolver": {"block": pblk, "degree": deg_c, "passes": passes_c, "residual": res_c, "rc": rc_c,
                                 "s": t_eig_c, "abs_re_lambda_min": float(np.abs(lamd.real).min()),
                                 "abs_re_lambda_max": float(np.abs(lamd.real).max())},
                 "nested_err_deflated": e_defl, "nested_err_undeflated": eps_nested,
                 "reference": f"non-nested k={kref}",
                 "smallest_k_at_target_deflated": k_defl, "k_grid": "300..k step 50",
                 "ms_per_apply": t_d * 1e3, "applies_per_s": 1.0 / t_d,
                 "applies_per_s_at_smallest_k": (1.0 / t_dk) if t_dk else None,
                 "overhead_ms": t_over * 1e3, "algorithmic_bytes": defl_bytes,
                 "overhead_GBps": defl_bytes / max(t_over, 1e-9) / 1e9}
    del rd, ld

    # the Hermitian eigensolver for deflation at mu = 0 on the same lattice:
    # the 16 eigenpairs of gamma5 Dw(0) smallest in modulus, then the nested
    # sign at mu = 0 (same k, l) with and without them, against a
    # non-nested reference at k = 1000
    m_e, p_e, deg_e = 16, 32, 40
    V0 = torch.from_numpy(latgen.random_sources(DIMS, p_e, 11).reshape(-1)).to(dev)
    R_e = torch.empty(m_e * 12 * DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3], dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam_e, passes_e, res_e, rc_e = nk.nk_eig_hermitian_device(lat.h, M_W, m_e, p_e, deg_e, 1e-10, 100, V0, R_e)
    t_e = time.perf_counter() - t0
    del V0
    p0 = nk.nk_sign_params_default(k=1000, ell=0, mu=0.0, m_w=M_W)
    y0ref = torch.empty_like(x)
    nk.nk_sign_apply_device(lat.h, p0, x, y0ref)
    p0 = nk.nk_sign_params_default(k=args.k, ell=args.ell, mu=0.0, m_w=M_W)
    nk.nk_sign_apply_device(lat.h, p0, x, y)
    e_none = rel(y, y0ref)
    nk.nk_sign_apply_deflated_device(lat.h, p0, lam_e.astype(np.complex128), R_e, R_e, x, y)
    e_defl = rel(y, y0ref)
    eig_mu0 = {"m": m_e, "block": p_e, "degree": deg_e, "passes": passes_e, "residual": res_e, "rc": rc_e,
               "s": t_e, "abs_lambda_min": float(np.abs(lam_e).min()), "abs_lambda_max": float(np.abs(lam_e).max()),
               "nested_mu0_err_undeflated": e_none, "nested_mu0_err_deflated": e_defl,
               "k": args.k, "ell": args.ell, "reference": "non-nested k=1000, mu=0"}
    del R_e, y0ref

    # the overlap operator of Eq. (1) in a linear solve: CGNR for Dov y = b at
    # the same (k, l), two sign applications per iteration; the true residual
    # is checked with one more application
    b_ov = torch.from_numpy(latgen.random_sources(DIMS, 1, 8)[0].reshape(-1)).to(dev)
    y_ov = torch.empty_like(b_ov)
    r_ov = torch.empty_like(b_ov)
    p_ov = params(args.k, args.ell, scaling=LEARNED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_ov, res_ov, rc_ov = nk.nk_overlap_solve_device(lat.h, p_ov, 1e-7, 200, b_ov, y_ov)
    torch.cuda.synchronize()
    t_ov = time.perf_counter() - t0
    nk.nk_overlap_apply_device(lat.h, p_ov, False, y_ov, r_ov)
    overlap_solve = {"solver": "CGNR on Dov(mu) y = b", "tol": 1e-7, "k": args.k, "ell": args.ell,
                     "iterations": it_ov, "recursive_residual": res_ov, "rc": rc_ov,
                     "true_residual": rel(r_ov, b_ov), "ms": t_ov * 1e3,
                     "ms_per_iteration": t_ov * 1e3 / max(it_ov, 1),
                     "sign_applications": 2 * it_ov + 1}
    del b_ov, y_ov, r_ov

    # the double pass (Sec. 4): the basis is not stored, and a second pass
    # regenerates the right vectors with A alone from the stored coefficients
    # while accumulating the lift; its cost against the first pass
    p_one = params(args.k, args.ell, scaling=LEARNED)
    p_one.two_pass = nk.NK_TWO_PASS_OFF
    y_one = torch.empty_like(x)
    nk.nk_sign_apply_device(lat.h, p_one, x, y_one)
    pt = params(args.k, args.ell, scaling=LEARNED)
    pt.two_pass = nk.NK_TWO_PASS_ON
    nk.nk_sign_apply_device(lat.h, pt, x, y)
    t2 = []
    for _ in range(3):
        i2, _ = nk.nk_sign_apply_device(lat.h, pt, x, y)
        t2.append((i2.t_basis_ms, i2.t_lift_ms))
    two_pass = {"k": args.k, "ell": args.ell, "first_pass_ms": min(a for a, _ in t2),
                "second_pass_ms": min(b for _, b in t2), "rel_diff_vs_one_pass": rel(y, y_one),
                "second_pass": "right vectors regenerated with A alone from the stored coefficients, "
                               "lift accumulated as they appear"}
    del y_one

    # the non-nested small problem alone (Roberts-Higham on the dense k x k
    # Ritz matrix, Eq. (4)) at k = 500 and 1000, on H_k of this lattice:
    # the inversion-only iteration and the default with the Newton-Schulz
    # tail; every step is counted as 8 k^3 real flops, the k^3 complex
    # multiply-adds of a Gauss-Jordan inverse (a Newton-Schulz step's two
    # complex products are twice that, so the figure is a lower bound there),
    # against the 78.6 TFLOP/s FP64 peak
    rh_dense = {"lattice": "16^4", "mu": MU, "flops_per_step": "8 k^3", "peak_TFLOPs": 78.6}
    al_d, be_d, de_d, _, _ = nk.nk_krylov_basis_device(lat.h, nk.nk_sign_params_default(k=1000, mu=MU, m_w=M_W), x)
    for kd in (500, 1000):
        for ns_on in (False, True):
            nk.nk_rh_newton_schulz(ns_on)
            pd_ = nk.nk_sign_params_default()
            ts_ = []
            for _ in range(3):
                t0 = time.perf_counter()
                _, inf_d, _ = nk.nk_small_sign(kd, 0, False, al_d[:kd], be_d[:kd], de_d[:kd], pd_)
                ts_.append(time.perf_counter() - t0)
            tbest = min(ts_[1:])
            tf = inf_d.rh_iters * 8.0 * kd ** 3 / tbest / 1e12
            rh_dense[f"k{kd}_{'newton_schulz_tail' if ns_on else 'inversions_only'}"] = {
                "ms": tbest * 1e3, "steps": inf_d.rh_iters, "TFLOPs": tf, "frac_of_fp64_peak": tf / 78.6,
                "residual": inf_d.rh_residual}
    nk.nk_rh_newton_schulz(True)
    del al_d, be_d, de_d

    ng = nk.nk_stencil_groups(lat.h, nk.NK_PREC_FP64, False)
    V = DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3]

    # the two kernels of an outer step in every precision and recurrence:
    # HIP events on every launch of a short plain run (k = 60) on the same
    # lattice, after one untimed run (which also tunes the kernel)
    copy_gbs = copy_rate(torch, dev)
    streams = stream_ceiling(torch, nk, dev)
    step_kernels = {}
    for prec, pname in ((nk.NK_PREC_FP64, "fp64"), (nk.NK_PREC_FP32, "fp32"),
                        (nk.NK_PREC_FP32_BF16LINKS, "fp32_bf16links")):
        for mu, rname in ((MU, "two_sided"), (0.0, "lanczos")):
            pk = nk.nk_sign_params_default(k=60, ell=0, mu=mu, m_w=M_W, precision=prec, profile=1)
            nk.nk_sign_apply_device(lat.h, pk, x, y)
            info_k, _ = nk.nk_sign_apply_device(lat.h, pk, x, y)
            b1, b2 = step_kernel_bytes(mu == 0.0, prec)
            u1 = info_k.t_stencil_ms / max(info_k.n_stencil, 1) * 1e3
            u2 = info_k.t_update_ms / max(info_k.n_update, 1) * 1e3
            step_kernels[f"{pname}_{rname}"] = {
                "groups": nk.nk_stencil_groups(lat.h, prec, mu == 0.0),
                "k1_us": u1, "k1_bytes_per_site": b1, "k1_GBps": b1 * V / u1 / 1e3,
                "k2_us": u2, "k2_bytes_per_site": b2, "k2_GBps": b2 * V / u2 / 1e3,
            }
    for v in step_kernels.values():
        v["k1_frac_of_copy"] = v["k1_GBps"] / copy_gbs
        v["k1_frac_of_peak"] = v["k1_GBps"] / HBM_PEAK_GBS

    stencil = stencil_rates(torch, nk, latgen, dev, copy_gbs)

    # the precision workload at its parameters (k = 1000, l = 200): each
    # reduced-precision result against the FP64 one on the same source
    precision = {"lattice": "16^4", "k": 1000, "ell": 200}
    for mu_p in (0.0, MU):
        y64 = torch.empty_like(x)
        yp = torch.empty_like(x)
        nk.nk_sign_apply_device(lat.h, nk.nk_sign_params_default(k=1000, ell=200, mu=mu_p, m_w=M_W), x, y64)
        for prec, pname in ((nk.NK_PREC_FP32, "fp32"), (nk.NK_PREC_FP32_BF16LINKS, "fp32_bf16links")):
            nk.nk_sign_apply_device(lat.h, nk.nk_sign_params_default(k=1000, ell=200, mu=mu_p, m_w=M_W,
                                                                     precision=prec), x, yp)
            precision[f"{pname}_mu{mu_p}_rel_err_vs_fp64"] = rel(yp, y64)
        del y64, yp

    # the block stencil step: 32 sources in lockstep at 16^3 x 32 (plain,
    # k = 40), per source, beside the one-source kernel on the same lattice
    bdims, nsrc = (16, 16, 16, 32), 32
    Vb = bdims[0] * bdims[1] * bdims[2] * bdims[3]
    with nk.Lattice(bdims) as blat:
        nk.nk_gauge_set(blat.h, latgen.random_gauge(bdims, EPS, 0))
        xs = torch.from_numpy(latgen.random_sources(bdims, nsrc, 3).reshape(-1)).to(dev)
        ys = torch.empty_like(xs)
        p1 = nk.nk_sign_params_default(k=40, ell=0, mu=MU, m_w=M_W, profile=1)
        nk.nk_sign_apply_device(blat.h, p1, xs[:12 * Vb], ys[:12 * Vb])
        i1, _ = nk.nk_sign_apply_device(blat.h, p1, xs[:12 * Vb], ys[:12 * Vb])
        pbk = nk.nk_sign_params_default(k=40, ell=0, mu=MU, m_w=M_W, profile=1, nrhs=nsrc, block=1)
        nk.nk_sign_apply_device(blat.h, pbk, xs, ys)
        blk_choice = nk.nk_block_group(blat.h)
        per_group = {}
        for grp in (1, 2, 4):  # each group size forced in turn, then back to the tuner's choice
            nk.nk_block_group(blat.h, grp)
            nk.nk_sign_apply_device(blat.h, pbk, xs, ys)
            ig, _ = nk.nk_sign_apply_device(blat.h, pbk, xs, ys)
            per_group[str(grp)] = ig.t_stencil_ms / max(ig.n_stencil, 1) * 1e3 / nsrc
        nk.nk_block_group(blat.h, blk_choice)
        ibk, _ = nk.nk_sign_apply_device(blat.h, pbk, xs, ys)
        del xs, ys
        # the batching workload at full size: 32 sources with l uniform in
        # [40, 300] (seeded), k = 600, lockstep sweeps replayed from graphs.
        # The first application captures the graphs; the second, timed, is
        # applied to the first's result, so sgn(sgn x) = x measures the error
        xs = torch.from_numpy(latgen.random_sources(bdims, nsrc, 4).reshape(-1)).to(dev)
        ys, zs = torch.empty_like(xs), torch.empty_like(xs)
        ells4 = [int(e) for e in latgen.uneven_ell(nsrc, 40, 300, 0)]
        p4 = nk.nk_sign_params_default(k=600, mu=MU, m_w=M_W, nrhs=nsrc, block=2, ell_per_rhs=ells4,
                                       rh_scaling=LEARNED)
        nk.nk_sign_apply_device(blat.h, p4, xs, ys)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info4, _ = nk.nk_sign_apply_device(blat.h, p4, ys, zs)
        torch.cuda.synchronize()
        t4 = time.perf_counter() - t0
        nb4 = 12 * Vb
        r4 = max(float(torch.linalg.vector_norm(zs[i * nb4:(i + 1) * nb4] - xs[i * nb4:(i + 1) * nb4])
                       / torch.linalg.vector_norm(xs[i * nb4:(i + 1) * nb4])) for i in range(nsrc))
        batching = {"lattice": "16^3x32", "mu": MU, "eps": EPS, "sources": nsrc, "k": 600,
                    "ell_min": min(ells4), "ell_max": max(ells4), "scaling": "learned" if have_model else "none",
                    "ms_per_batch": t4 * 1e3, "sources_per_s": nsrc / t4, "two_pass": info4.two_pass,
                    "sgn_squared_residual_max": r4}
        del xs, ys, zs
    # the learned scaling away from the data it was trained on: H_l (l = 250)
    # of the inner projection at 24^4, mu = 0.5, link width 1.0, k = 1200,
    # for two sources; Roberts-Higham iterations with each scaling and the
    # largest |S^2 - 1|_F / sqrt(l) of the results
    ldims, lk, lell, lmu = (24, 24, 24, 24), 1200, 250, 0.5
    rh24 = {"lattice": "24^4", "mu": lmu, "eps": 1.0, "k": lk, "ell": lell, "sources": 2}
    mats = []
    with nk.Lattice(ldims) as llat:
        nk.nk_gauge_set(llat.h, latgen.random_gauge(ldims, 1.0, 0))
        lsrc = latgen.random_sources(ldims, 2, 5)
        for s_ in range(2):
            xl = torch.from_numpy(np.ascontiguousarray(lsrc[s_]).reshape(-1)).to(dev)
            al, be, de, info_l, _ = nk.nk_krylov_basis_device(
                llat.h, nk.nk_sign_params_default(k=lk, mu=lmu, m_w=M_W), xl)
            kk = info_l.k_used
            a_, b_, d_, _, _ = nk.nk_inner_matrix(kk, min(lell, kk), False, al[:kk], be[:kk], de[:kk])
            mats.append(rh_train.tridiag_dense(a_, b_, d_))
            del xl
    for name, sc in (("none", nk.NK_RH_NONE), ("det", nk.NK_RH_DET), ("learned", LEARNED)):
        its, res = [], 0.0
        for m in mats:
            out_m, it_m, _ = nk.nk_rh_sign(m[None], scaling=sc)
            its.append(int(it_m[0]))
            sq = out_m[0] @ out_m[0]
            res = max(res, float(np.linalg.norm(sq - np.eye(sq.shape[0])) / np.sqrt(sq.shape[0])))
        rh24[f"rh_iters_{name}"] = its
        rh24[f"resid_{name}"] = res
    one_us = i1.t_stencil_ms / max(i1.n_stencil, 1) * 1e3
    blk_us = ibk.t_stencil_ms / max(ibk.n_stencil, 1) * 1e3 / nsrc
    block_stencil = {
        "lattice": "16^3x32", "sources": nsrc, "k": 40,
        "k1_us_per_source": blk_us, "k1_GBps_per_source": K1_BYTES_PER_SITE * Vb / blk_us / 1e3,
        "one_source_k1_us": one_us, "one_source_k1_GBps": K1_BYTES_PER_SITE * Vb / one_us / 1e3,
        "k2_us_per_source": ibk.t_update_ms / max(ibk.n_update, 1) * 1e3 / nsrc,
        "sources_per_workgroup": blk_choice,
        "k1_us_per_source_by_group": per_group,
        "link_amortised_bytes_per_site_source": 1152 + 576 / blk_choice,
        "k1_GBps_link_amortised": (1152 + 576 / blk_choice) * Vb / blk_us / 1e3,
    }
    k1_avg_s = (t_st / max(n_st, 1)) / 1e3
    k1_bytes = K1_BYTES_PER_SITE * V
    achieved = k1_bytes / k1_avg_s / 1e9
    traffic = None
    if os.path.exists(PROFILE_PMC):
        with open(PROFILE_PMC) as fh:
            pmc = json.load(fh)
        if pmc.get("source_hash") == kernel_source_hash():
            traffic = pmc.get("bytes_per_launch")
    out = {
        "metric": "sgn(g5 Dw) x applies/sec at 16^4 mu=0.3, nested vs plain @1e-8; stencil HBM GB/s",
        "value": 1.0 / t_nested,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_nested * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "16^4 lattice, mu=0.3 two-sided Lanczos, m_w=-1, random SU(3) links eps=0.8 seed 0, "
                        "1 Gaussian source, nested sign with learned Roberts-Higham scaling at relative "
                        "accuracy 1e-8",
            "k": args.k,
            "ell": args.ell,
            "eps_nested": eps_nested,
            "eps_plain": eps_plain,
            "reference": f"non-nested k={kref}",
        },
        "forms": {
            "nested_learned": {"applies_per_s": 1.0 / t_nested, "rh_iters": rh_iters,
                               "small_ms": ph["small"] / args.steps},
            "nested_determinant": {"applies_per_s": 1.0 / t_nested_d, "rh_iters": info_d["rh_iters"],
                                   "small_ms": info_d["t_small_ms"] / args.steps},
            "nested_unscaled": {"applies_per_s": 1.0 / t_nested_u, "rh_iters": info_u["rh_iters"],
                                "small_ms": info_u["t_small_ms"] / args.steps},
            "plain_unscaled": {"applies_per_s": 1.0 / t_plain, "rh_iters": info_p["rh_iters"],
                               "small_ms": info_p["t_small_ms"] / args.steps},
            f"nested_learned_batched_{nb}": {"applies_per_s_per_source": nb / t_batch, "ms_per_batch": t_batch * 1e3,
                                             "two_pass": info_b.two_pass},
        },
        "forms_interleaved": forms_interleaved,
        "nested_vs_plain_speedup": t_plain / t_nested,
        "rh_inverse_shape_k": nk.nk_rh_tile_choice(args.k, 1),
        "learned_model": os.path.relpath(rh_train.WEIGHTS, ROOT) if have_model else None,
        "phases_ms": {k: v / args.steps for k, v in ph.items()},
        "rh_iters": rh_iters,
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_bil1<double, LinksPlain<double>, {ng}> (fused A v, A^dag w two-sided Lanczos stencil "
                      f"step, FP64, {ng} direction groups chosen by the autotuner)",
            "sampled": f"HIP events on the kernels of every {PROFILE_EVERY}th outer step of the timed applications",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            # the counted traffic per launch over the same launch time, beside
            # the fastest of this run's own streaming kernels
            "traffic_GBps": traffic / k1_avg_s / 1e9 if traffic else None,
            "stream_ceiling_GBps": max((v["GBps"] for v in streams.values() if isinstance(v, dict) and "GBps" in v),
                                       default=None),
            "avg_launch_us": k1_avg_s * 1e6,
            "launches": int(n_st),
            "bytes_per_launch": k1_bytes,
        },
        "update_kernel": {"avg_launch_us": (t_up / max(n_up, 1)) * 1e3, "launches": int(n_up)},
        "copy_GBps": copy_gbs,
        "stream_ceiling": streams,
        "step_kernels": step_kernels,
        "stencil": stencil,
        "precision_vs_fp64": precision,
        "block_stencil": block_stencil,
        "batching_16x16x16x32": batching,
        "learned_scaling_24x24x24x24": rh24,
        "rh_dense": rh_dense,
        "two_pass": two_pass,
        "deflation": deflation,
        "overlap_solve": overlap_solve,
        "eigensolver_mu0": eig_mu0,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.k, args.ell, args.cpu_sample_steps)
    lat.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
