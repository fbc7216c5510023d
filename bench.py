"""Benchmark of the sum-factorized Helmholtz operator and its solvers on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Default workload `helmholtz_p4_32e` (32^3 hexes, p = 4, q = 6, 2.1M DoFs, alpha = 1e3,
beta = 1, nu(x) = 1 + 0.5 sin(2 pi x) cos(2 pi y)).  One timed step = one FP64 Helmholtz
apply y = (alpha M + beta K(nu)) x over the whole workload (gather, three
contractions, quadrature function, three transposed contractions, atomic-free
assembly).  `value` is that apply's throughput in GDoF/s (global DoFs per second)
with every input resident in HBM.  The same run times the FP32 apply, the FP64
Jacobi-PCG solve and the FP32-inner iterative-refinement solve to relative residual
1e-10, and the adjoint gradient kernel; the CPU oracle is timed on a bounded sample of
the same workload.  Prints one JSON line.

Other workloads (`--workload`): vector_helmholtz_p7_24e, adjoint_p5_20e, large_p8_40e,
stokes_32e (Taylor-Hood block operator apply, 32^3 hexes, p = 2..6), convection (the
N(u) term for p = 1..8 on 1.8-4.8M DoFs per component),
poisson_p2_4e, `sweep` (FP64/FP32 apply for p = 4..8 on meshes of 15-33M DoFs),
`mass_neumann` (collocated-mass-preconditioned mass solve and pure-Neumann Poisson solve),
`projection_32e` (projection time steps), `lor_p4_32e` (the LOR multigrid preconditioner
against Jacobi) and `lor_sweep` (the LOR-preconditioned pure-Neumann solve for p = 2..8 on
~2.1M DoFs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s of sum-factorized Helmholtz apply (FP64 vs FP32+IR); PCG time to 1e-10"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 vector
SWEEP = [(4, 64), (5, 50), (6, 45), (7, 40), (8, 40)]  # (p, elements per direction)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="helmholtz_p4_32e")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the p = 4..8 sweep and the three-member p = 7 apply of the default line")
    ap.add_argument("--sets", type=int, default=4,
                    help="independent operator/vector copies cycled by the timed applies")
    ap.add_argument("--cpu-elements", type=int, default=32768,
                    help="upper bound on the elements the CPU oracle applies (sample sized to ~15 s)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MB (hardware-counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM bytes of one FP64 Helmholtz apply on the metric's workload (element kernel +
# assembly dispatch), from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a plain
# copy's readings; valid only for the kernel sources they were taken with (keyed by
# the hash of those sources), otherwise the roofline reports traffic = null.
KERNEL_SOURCES = ["apply_impl.h", "eo.h", "rules.h", "internal.h", "plan.h", "k_apply_f64.hip", "k_vec.hip"]
MEASURED_TRAFFIC = {
    # profiles/helmholtz_apply_p4_32e_hbm_bytes.md (FP64 apply, both dispatches)
    ("a7986bae1c3cc88f", "helmholtz_p4_32e"): 553476720,
    # profiles/vector_helmholtz_p7_24e_counters.md (three-member FP64 apply)
    ("a7986bae1c3cc88f", "vector_helmholtz_p7_24e"): 1288660473,
}
# Executed floating-point operations of one apply (element kernel + assembly) from the
# SQ_INSTS_VALU_FLOPS_FP64 / _FP32 counters (x 64 lanes), same keying as the traffic:
# profiles/helmholtz_apply_p4_32e_counters.md, profiles/vector_helmholtz_p7_24e_counters.md.
MEASURED_FLOPS = {
    ("a7986bae1c3cc88f", "helmholtz_p4_32e"): {"fp64": 961714752, "fp32": 964111936},
    ("a7986bae1c3cc88f", "vector_helmholtz_p7_24e"): {"fp64": 6564470208, "fp32": 6260121024},
}
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 vector


def code_of(text):
    """Source text without // comments and blank lines (a comment edit is not a kernel
    change)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code.strip():
            out.append(code)
    return "\n".join(out)


def kernel_source_hash(read=None):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, "paper_1910_03032_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(code_of(text).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(nelem, p, ndof, s, nb=1, nqd=7, nb_qd=1):
    """Bytes an apply must move: quadrature data once (per distinct field), x read and
    y written once per member, the element->DoF map once."""
    q = p + 2
    return nb_qd * nelem * q ** 3 * nqd * s + nb * 2 * ndof * s + nelem * (p + 1) ** 3 * 4


def flops_helmholtz(nelem, p, nb=1):
    n, q = p + 1, p + 2
    return nelem * nb * (2 * (4 * q * n ** 3 + 6 * q * q * n * n + 8 * q ** 3 * n) + 25 * q ** 3)


def counter_rate(workload, prec, ms):
    """Counter-measured flops of one apply of `workload` (keyed by the kernel sources) over
    `ms` milliseconds, in TFLOP/s; None when the sources differ from the measured ones."""
    f = MEASURED_FLOPS.get((kernel_source_hash(), workload))
    return None if f is None else round(f[prec] / (ms * 1e-3) / 1e12, 2)


def counter_frac(workload, prec, ms, peak_tflops):
    r = counter_rate(workload, prec, ms)
    return None if r is None else round(r / peak_tflops, 4)


def copy_calibration(mb, reps=5):
    """A plain device-to-device copy of known size: reference for the HBM byte counters."""
    import torch
    n = mb * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps,
                      "us": round(ms * 1e3, 1), "GBps": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}),
          flush=True)
    return 0


class Bench:
    """One workload on the GPU.  `nsets` independent copies of the operator (quadrature
    data, map, E-vector) and of x, y are applied in turn, so that a working set smaller
    than the 256 MB last-level cache is not served from that cache on repeats."""

    def __init__(self, ne, p, alpha, beta, nu="c2", nsets=1):
        import torch
        from paper_1910_03032_amd import Operator
        from workloads import BoxMesh, nu_c2
        self.torch = torch
        self.dev = torch.device("cuda", 0)
        t0 = time.time()
        self.m = m = BoxMesh(ne, p)
        self.ne, self.p, self.q, self.alpha, self.beta = ne, p, p + 2, alpha, beta
        self.ops = []
        for _ in range(max(1, nsets)):
            op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=m.ess)
            if nu == "c2":
                xq = op.qpoint_coords()
                op.set_coeffs(alpha, beta, nu_c2(xq[0], xq[1], xq[2]))
                del xq
            else:
                op.set_coeffs(alpha, beta, None)
            self.ops.append(op)
        self.op = self.ops[0]
        self.info = self.op.info()
        self.stream = torch.cuda.current_stream(self.dev)
        log(f"[bench] setup {time.time() - t0:.1f}s: {ne}^3 p={p} ndof={m.ndof} "
            f"device bytes={self.info['device_bytes'] / 1e9:.2f} GB x {len(self.ops)} set(s)")

    def close(self):
        for op in self.ops:
            op.close()
        self.ops = []

    @staticmethod
    def timed_fn(fn, steps, warmup):
        """Average ms of fn over `steps` calls after `warmup`, HIP events on the current stream."""
        import torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        st = torch.cuda.current_stream()
        e0.record(st)
        for _ in range(steps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def timed(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(steps):
            fn()
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms

    def apply_rate(self, dtype, nb=1, steps=50, warmup=10):
        """Time `steps` applies, cycling over the operator copies; inputs are resident."""
        from paper_1910_03032_amd import HELMHOLTZ
        from workloads import normal
        torch = self.torch
        N = self.m.ndof
        k = len(self.ops)
        xs, ys = [], []
        for i in range(k):
            x = torch.as_tensor(normal(nb * N, seed=1 + i), device=self.dev)
            x = (x.reshape(nb, N) if nb > 1 else x).to(dtype)
            xs.append(x)
            ys.append(torch.empty_like(x))
        it = [0]

        def step():
            i = it[0] % k
            self.ops[i].apply(xs[i], op=HELMHOLTZ, out=ys[i])
            it[0] += 1

        ms = self.timed(step, steps, warmup)
        s = 8 if dtype == torch.float64 else 4
        nbytes = algorithmic_bytes(self.m.nelem, self.p, N, s, nb=nb)
        return {"us": round(ms * 1e3, 2), "GDoF/s": round(nb * N / (ms * 1e-3) / 1e9, 3),
                "algorithmic_GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "algorithmic_bytes": nbytes, "buffer_sets": k}

    def solve(self, b, mode, reps=3, **kw):
        torch = self.torch
        best, res, xs = None, None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            xs, res = self.op.pcg(b, rtol=1e-10, mode=mode, inner_rtol=1e-5, check_every=16, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        return xs, {"ms": round(best * 1e3, 2), "iters": res.iters, "outer": res.outer,
                    "true_rel_res": res.true_rel_res, "status": res.status}


def host_cpu():
    """Host CPU of this run: logical CPU count, model name, BLAS threads in use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        blas = None
    return {"cpu_count": os.cpu_count(), "model": model, "blas_threads": blas}


def cpu_baseline(m, p, alpha, beta, max_elements, target_s=12.0):
    """The oracle's dense (non-sum-factorized) FP64 apply on the first elements of the
    workload, with the BLAS threads the host gives (a 1024-element probe sizes the sample
    to about `target_s` seconds) and with one thread (a 1024-element sample); plus the
    oracle's Jacobi-PCG Poisson solve of the 4^3, p = 2 workload to 1e-10."""
    from oracle import Discretization, pcg
    from workloads import nu_c2, normal, BoxMesh, rhs_uniform
    host = host_cpu()
    x = normal(m.ndof, seed=1)

    used = [1.0]

    def run(sub):
        d = Discretization(m.elem_xyz[:sub], m.elem_dofs[:sub], m.ess, m.ndof, p, p + 2)
        xq = d.qpoint_coords()
        nu = nu_c2(xq[..., 0], xq[..., 1], xq[..., 2])
        t, c = time.perf_counter(), time.process_time()
        d.apply_unconstrained(x, alpha, beta, nu)
        wall = time.perf_counter() - t
        used[0] = (time.process_time() - c) / max(wall, 1e-9)  # CPU seconds per second
        return wall

    probe = min(1024, m.nelem, max_elements)
    dt = run(probe)
    sub = int(min(max_elements, m.nelem, max(probe, probe * target_s / max(dt, 1e-3))))
    if sub > probe:
        dt = run(sub)
    dofs = m.ndof * sub / m.nelem
    cores = max(1, int(round(used[0])))
    log(f"[bench] cpu oracle: {sub} elements in {dt:.2f}s ({host['blas_threads']} BLAS threads, "
        f"{used[0]:.1f} cores busy)")
    out = {"value": round(dofs / dt / 1e9, 7), "unit": "GDoF/s", "cores": cores,
           "kind": "oracle",
           "sample": f"dense FP64 element apply over {sub} of {m.nelem} elements "
                     f"({dt:.2f} s), DoFs scaled by the element fraction; cores = CPU time / wall "
                     f"time of the sample ({used[0]:.2f}) with {host['blas_threads']} BLAS threads allowed",
           "host": host}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            d1 = run(probe)
        out["one_thread"] = {"value": round(m.ndof * probe / m.nelem / d1 / 1e9, 7), "unit": "GDoF/s",
                             "sample": f"{probe} elements in {d1:.2f} s"}
        log(f"[bench] cpu oracle, 1 thread: {probe} elements in {d1:.2f}s")
    except Exception as e:  # threadpoolctl missing or unable to limit
        out["one_thread"] = {"error": str(e)}
    # the oracle's PCG on the 4^3, p = 2 Poisson workload (element-matrix applies)
    mc = BoxMesh(4, 2)
    dc = Discretization(mc.elem_xyz, mc.elem_dofs, mc.ess, mc.ndof, 2, 4)
    bc = rhs_uniform(mc, seed=1)[0]
    dinv = 1.0 / dc.diagonal(0.0, 1.0)
    t = time.perf_counter()
    _, it, rr = pcg(lambda v: dc.apply(v, 0.0, 1.0), bc, dinv, rtol=1e-10)
    out["pcg_poisson_p2_4e"] = {"ms": round((time.perf_counter() - t) * 1e3, 2), "iters": it,
                                "rel_res": rr, "ndof": mc.ndof}
    return out


def run_main(a, wl):
    """The metric's configuration: FP64 apply as the timed step, plus solves."""
    from workloads import rhs_uniform
    torch = __import__("torch")
    B = Bench(wl["ne"], wl["p"], wl["alpha"], wl["beta"], nsets=a.sets)
    m, p, q, N = B.m, B.p, B.q, B.m.ndof
    r64 = B.apply_rate(torch.float64, steps=a.steps, warmup=a.warmup)
    log(f"[bench] fp64 apply {r64['us']} us  {r64['GDoF/s']} GDoF/s")
    r32 = B.apply_rate(torch.float32, steps=a.steps, warmup=a.warmup)
    log(f"[bench] fp32 apply {r32['us']} us  {r32['GDoF/s']} GDoF/s")
    ms64 = r64["us"] * 1e-3
    achieved = r64["algorithmic_bytes"] / (ms64 * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": r64["GDoF/s"],
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms64, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded perturbed hex mesh, x ~ N(0,1))",
        "config": {"workload": a.workload, "elements": f"{B.ne}^3", "p": p, "q": q, "ndof": N,
                   "alpha": B.alpha, "beta": B.beta,
                   "nu": "1+0.5 sin(2 pi x) cos(2 pi y) at quadrature points",
                   "step": "one FP64 Helmholtz apply"},
        # one apply = the element kernel + the assembly kernel, on one stream
        "roofline": {
            "bound": "hbm",
            "kernel": f"Helmholtz apply: apply_kernel<{p}, double, 2> + assemble_kernel<double>",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_TRAFFIC.get((kernel_source_hash(), a.workload)),
            "traffic_unit": "HBM bytes per apply (both dispatches)",
            "kernel_source_hash": kernel_source_hash(),
            "algorithmic_bytes_per_apply": r64["algorithmic_bytes"],
            "launches_per_apply": 2,
            "apply_us": r64["us"],
            # executed FP64 flops from the counters (null once the kernel sources change)
            # over the live apply time, against the 78.6 TFLOP/s FP64 peak
            "fp64_flop_rate_tflops": counter_rate("helmholtz_p4_32e", "fp64", ms64),
            "fp64_flop_frac": counter_frac("helmholtz_p4_32e", "fp64", ms64, FP64_PEAK_TFLOPS),
            "fp64_model_flop_rate_tflops": round(flops_helmholtz(m.nelem, p) / (ms64 * 1e-3) / 1e12, 2),
        },
        "fp32_apply": dict(r32, value=r32["GDoF/s"], unit="GDoF/s",
                           fp32_flop_rate_tflops=counter_rate("helmholtz_p4_32e", "fp32", r32["us"] * 1e-3),
                           note=f"{r32['buffer_sets']} operator/vector sets of "
                                f"{r32['algorithmic_bytes'] / 1e6:.0f} MB applied in turn "
                                f"({r32['buffer_sets'] * r32['algorithmic_bytes'] / 1e6:.0f} MB), so "
                                "a repeat is not served from the 256 MB last-level cache"),
    }
    if not a.no_solves:
        b = torch.as_tensor(rhs_uniform(m, seed=1)[0], device=B.dev)
        xs, s64 = B.solve(b, 0)
        log(f"[bench] pcg fp64 {s64}")
        _, sir = B.solve(b, 1)
        log(f"[bench] pcg fp32+IR {sir}")
        out["pcg_fp64"] = s64
        out["pcg_fp32_ir"] = sir
        out["ir_speedup"] = round(s64["ms"] / sir["ms"], 3)
        lam = xs.clone()
        msg = B.timed(lambda: B.op.grad_nu(xs, lam), 10, 2)
        gbytes = m.nelem * q ** 3 * 6 * 8 + 2 * N * 8 + m.nelem * q ** 3 * 8 + m.nelem * (p + 1) ** 3 * 4
        out["adjoint_grad_kernel"] = {"us": round(msg * 1e3, 1),
                                      "algorithmic_GBps": round(gbytes / (msg * 1e-3) / 1e9, 1)}
    if not a.no_sweep:
        # the >= 60 % target's evidence, timed in the same run: FP64 / FP32 applies at
        # p = 4..8 on 15-33M DoF meshes (one operator copy each: 1.4-4.3 GB per apply, far
        # above the last-level cache), and the three-member p = 7 apply
        B.close()
        del B
        torch.cuda.empty_cache()
        out["sweep_p4_8"] = run_sweep(a, steps=10, warmup=2)["rows"]
        out["vector_helmholtz_p7_24e"] = vector_apply_rates(a, WORKLOADS_VECTOR)
        torch.cuda.empty_cache()
        if not a.no_solves:
            # the flow solver's timings in the same run: the pressure Poisson solve with the
            # LOR preconditioner, and one projection time step with the stepper's defaults
            from paper_1910_03032_amd import PRECOND_LOR32
            from workloads import BoxMesh
            out["lor_neumann_poisson_p4_32e"] = lor_poisson_row()
            out["projection_step_p4_32e"] = projection_row(a, BoxMesh(32, 4), 32, 4,
                                                           "lor_fp32_vcycle_velocity_ir",
                                                           PRECOND_LOR32, 0, 1)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, p, wl["alpha"], wl["beta"], a.cpu_elements)
    return out


WORKLOADS_VECTOR = "vector_helmholtz_p7_24e"


def vector_apply_rates(a, name):
    """FP64 and FP32 applies of the three-member Helmholtz workload (24^3, p = 7), one
    operator copy (824 MB per FP64 apply): GDoF/s over the 3 N DoFs, the HBM fraction of
    the algorithmic bytes and the model FP64 flop rate."""
    torch = __import__("torch")
    from workloads import WORKLOADS
    wl = WORKLOADS[name]
    B = Bench(wl["ne"], wl["p"], wl["alpha"], wl["beta"], nsets=1)
    nb = wl["nbatch"]
    r64 = B.apply_rate(torch.float64, nb=nb, steps=10, warmup=2)
    r32 = B.apply_rate(torch.float32, nb=nb, steps=10, warmup=2)
    fl = flops_helmholtz(B.m.nelem, B.p, nb)
    r64["fp64_model_tflops"] = round(fl / (r64["us"] * 1e-6) / 1e12, 2)
    r64["fp64_model_frac"] = round(fl / (r64["us"] * 1e-6) / 1e12 / FP64_PEAK_TFLOPS, 4)
    r64["fp64_flop_rate_tflops"] = counter_rate(name, "fp64", r64["us"] * 1e-3)
    r64["fp64_flop_frac"] = counter_frac(name, "fp64", r64["us"] * 1e-3, FP64_PEAK_TFLOPS)
    r64["traffic"] = MEASURED_TRAFFIC.get((kernel_source_hash(), name))
    r32["fp32_flop_rate_tflops"] = counter_rate(name, "fp32", r32["us"] * 1e-3)
    r32["fp32_flop_frac"] = counter_frac(name, "fp32", r32["us"] * 1e-3, FP32_PEAK_TFLOPS)
    log(f"[bench] {name}: fp64 {r64['us']} us ({r64['hbm_frac']:.3f} of HBM, "
        f"{r64['fp64_model_frac']:.3f} of FP64), fp32 {r32['us']} us")
    B.close()
    del B
    torch.cuda.empty_cache()
    return {"elements": f"{wl['ne']}^3", "p": wl["p"], "components": nb, "fp64": r64, "fp32": r32}


def run_vector(a, wl):
    """3-component Helmholtz: batched apply and FP64 PCG vs FP32-inner IR to 1e-10."""
    from workloads import rhs_uniform
    torch = __import__("torch")
    B = Bench(wl["ne"], wl["p"], wl["alpha"], wl["beta"], nsets=a.sets)
    nb = wl["nbatch"]
    out = {"workload": a.workload, "p": B.p, "elements": f"{B.ne}^3", "ndof_per_component": B.m.ndof,
           "components": nb,
           "apply_fp64": B.apply_rate(torch.float64, nb=nb, steps=a.steps, warmup=a.warmup),
           "apply_fp32": B.apply_rate(torch.float32, nb=nb, steps=a.steps, warmup=a.warmup)}
    if a.no_solves:
        return out
    b = torch.as_tensor(rhs_uniform(B.m, seed=1, nbatch=nb), device=B.dev)
    x64, out["pcg_fp64"] = B.solve(b, 0, reps=2)
    xir, out["pcg_fp32_ir"] = B.solve(b, 1, reps=2)
    out["ir_speedup"] = round(out["pcg_fp64"]["ms"] / out["pcg_fp32_ir"]["ms"], 3)
    out["ir_vs_fp64_solution_rel_diff"] = float((xir - x64).norm() / x64.norm())
    return out


def run_adjoint(a, wl):
    """Forward solve, adjoint solve and gradient kernel for nu ~ U(0.5, 2) per point."""
    from workloads import rhs_uniform, nu_uniform
    torch = __import__("torch")
    B = Bench(wl["ne"], wl["p"], wl["alpha"], wl["beta"], nu=None)
    m, op = B.m, B.op
    nu = torch.as_tensor(nu_uniform(m.nelem, B.q, seed=2), device=B.dev)
    nu_star = torch.as_tensor(nu_uniform(m.nelem, B.q, seed=3), device=B.dev)
    b = torch.as_tensor(rhs_uniform(m, seed=1)[0], device=B.dev)
    ess = torch.as_tensor(m.ess.astype(bool), device=B.dev)
    op.set_coeffs(B.alpha, B.beta, nu_star)
    u_t, _ = op.pcg(b, rtol=1e-12)
    torch.cuda.synchronize()
    t = time.perf_counter()
    op.set_coeffs(B.alpha, B.beta, nu)
    u, r1 = op.pcg(b, rtol=1e-10, check_every=16)
    lam, r2 = op.pcg(torch.where(ess, torch.zeros_like(u), u - u_t), rtol=1e-10, check_every=16)
    g = op.grad_nu(u, lam)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    msg = B.timed(lambda: op.grad_nu(u, lam), 10, 2)
    return {"workload": a.workload, "p": B.p, "elements": f"{B.ne}^3", "ndof": m.ndof,
            "gradient_total_ms": round(dt * 1e3, 2), "forward_iters": r1.iters[0],
            "adjoint_iters": r2.iters[0], "grad_kernel_us": round(msg * 1e3, 1),
            "grad_norm": float(g.norm())}


def run_large(a, wl):
    """p = 8, 33M DoFs: FP32+IR vs FP64 PCG to 1e-10, and the 4-field batched gradient."""
    from workloads import rhs_uniform, nu_uniform
    torch = __import__("torch")
    B = Bench(wl["ne"], wl["p"], wl["alpha"], wl["beta"])
    m, op = B.m, B.op
    out = {"workload": a.workload, "p": B.p, "elements": f"{B.ne}^3", "ndof": m.ndof,
           "apply_fp64": B.apply_rate(torch.float64, steps=20, warmup=3),
           "apply_fp32": B.apply_rate(torch.float32, steps=20, warmup=3)}
    b = torch.as_tensor(rhs_uniform(m, seed=1)[0], device=B.dev)
    _, out["pcg_fp64"] = B.solve(b, 0, reps=1)
    _, out["pcg_fp32_ir"] = B.solve(b, 1, reps=1)
    out["ir_speedup"] = round(out["pcg_fp64"]["ms"] / out["pcg_fp32_ir"]["ms"], 3)
    log(f"[bench] large solves {out['pcg_fp64']} {out['pcg_fp32_ir']}")
    nus = torch.stack([torch.as_tensor(nu_uniform(m.nelem, B.q, seed=200 + k).reshape(-1), device=B.dev)
                       for k in range(4)])
    ess = torch.as_tensor(m.ess.astype(bool), device=B.dev)
    B4 = b.expand(4, -1).contiguous()
    torch.cuda.synchronize()
    t = time.perf_counter()
    op.set_coeffs(B.alpha, B.beta, nus)
    U, r1 = op.pcg(B4, rtol=1e-10, mode=1, check_every=16)
    L, r2 = op.pcg(torch.where(ess, torch.zeros_like(U), U), rtol=1e-10, mode=1, check_every=16)
    G = op.grad_nu(U, L)
    torch.cuda.synchronize()
    out["batched_gradient_4_fields"] = {"ms": round((time.perf_counter() - t) * 1e3, 1),
                                        "forward_inner_iters": r1.iters, "adjoint_inner_iters": r2.iters,
                                        "forward_outer": r1.outer, "adjoint_outer": r2.outer,
                                        "forward_true_rel_res": r1.true_rel_res,
                                        "adjoint_true_rel_res": r2.true_rel_res,
                                        "converged": bool(r1.converged and r2.converged),
                                        "grad_norms": [float(G[k].norm()) for k in range(4)]}
    if not (r1.converged and r2.converged):
        raise RuntimeError(f"4-field batched solves did not converge: {r1} {r2}")
    return out


def run_mass_neumann(a):
    """The other two solves of a projection step at 32^3, p = 4 (no essential DoFs): the
    mass solve with the collocated mass preconditioner, and the pure-Neumann pressure
    Poisson solve (orthogonalized Jacobi-PCG, mean-zero solution), both to 1e-10."""
    import torch
    from paper_1910_03032_amd import Operator, MASS, DIFFUSION, PRECOND_COLLOCATED_MASS
    from workloads import BoxMesh, uniform
    m = BoxMesh(32, 4)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, 4)
    op.set_coeffs(0.0, 1.0, None)
    b = torch.as_tensor(uniform(m.ndof, seed=1), device="cuda")  # U(-1, 1) at every DoF

    def timed_solve(reps=3, **kw):
        best, res = None, None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, res = op.pcg(b, rtol=1e-10, check_every=16, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        return {"ms": round(best * 1e3, 2), "iters": res.iters, "outer": res.outer,
                "true_rel_res": res.true_rel_res, "status": res.status}

    out = {"workload": "mass_and_neumann_p4_32e", "p": 4, "elements": "32^3", "ndof": m.ndof,
           "mass_fp64_collocated": timed_solve(op=MASS, precond=PRECOND_COLLOCATED_MASS),
           "mass_fp32_ir_collocated": timed_solve(op=MASS, precond=PRECOND_COLLOCATED_MASS, mode=1),
           "mass_fp64_jacobi": timed_solve(op=MASS),
           "neumann_poisson_fp64": timed_solve(op=DIFFUSION, nullspace=True)}
    op.close()
    return out


def timed_solve(op, b, opk, **kw):
    """Best of two PCG solves to 1e-10 (wall time around the call, synchronized)."""
    import torch
    best, res = None, None
    for _ in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, res = op.pcg(b, op=opk, rtol=1e-10, check_every=16, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        best = dt if best is None else min(best, dt)
    return {"ms": round(best * 1e3, 2), "iters": res.iters, "true_rel_res": res.true_rel_res,
            "status": res.status}


def lor_poisson_row():
    """The projection step's pressure solve alone: the pure-Neumann Poisson problem on
    32^3 hexes at p = 4 to 1e-10, CG preconditioned by the LOR V-cycle in FP32 arithmetic
    against Jacobi."""
    import torch
    from paper_1910_03032_amd import DIFFUSION, PRECOND_LOR32, Operator
    from workloads import BoxMesh, uniform
    m = BoxMesh(32, 4)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, 4, ess=np_zeros(m.ndof))
    op.set_coeffs(0.0, 1.0, None)
    b = torch.as_tensor(uniform(m.ndof, seed=1), device="cuda")
    info = op.lor_setup(DIFFUSION)
    row = {"elements": "32^3", "p": 4, "ndof": m.ndof, "lor_levels": info["rows"],
           "lor_setup_ms": round(info["setup_ms"], 1),
           "pcg_lor_fp32_vcycle": timed_solve(op, b, DIFFUSION, precond=PRECOND_LOR32, nullspace=True),
           "pcg_jacobi": timed_solve(op, b, DIFFUSION, nullspace=True)}
    row["lor_speedup"] = round(row["pcg_jacobi"]["ms"] / row["pcg_lor_fp32_vcycle"]["ms"], 2)
    log(f"[bench] lor neumann_poisson (default line): {row}")
    op.close()
    return row


def run_lor(a):
    """The LOR preconditioner (Section 5.2) at 32^3, p = 4: host setup time and levels of
    the multigrid on A_LOR, the time of one V-cycle, and CG to 1e-10 preconditioned by it
    against Jacobi for the pure-Neumann Poisson problem (the projection step's pressure
    solve) and the Helmholtz workload (alpha = 1e3, beta = 1, nu(x) of the metric)."""
    import torch
    from paper_1910_03032_amd import DIFFUSION, F32, HELMHOLTZ, PRECOND_LOR, PRECOND_LOR32, Operator
    from workloads import BoxMesh, nu_c2, rhs_uniform, uniform
    m = BoxMesh(32, 4)
    out = {"workload": "lor_p4_32e", "p": 4, "elements": "32^3", "ndof": m.ndof}

    solve = timed_solve
    for name, ess, opk in (("neumann_poisson", np_zeros(m.ndof), DIFFUSION), ("helmholtz", m.ess, HELMHOLTZ)):
        op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, 4, ess=ess)
        if opk == HELMHOLTZ:
            xq = op.qpoint_coords()
            op.set_coeffs(1e3, 1.0, nu_c2(xq[0], xq[1], xq[2]))
            b = torch.as_tensor(rhs_uniform(m, seed=1)[0], device="cuda")
        else:
            op.set_coeffs(0.0, 1.0, None)
            b = torch.as_tensor(uniform(m.ndof, seed=1), device="cuda")
        info = op.lor_setup(opk)
        ms_v = Bench.timed_fn(lambda: op.lor_vcycle(b, opk), 10, 2)
        op.lor_vcycle(b, opk, prec=F32)  # makes the FP32 copies
        ms_v32 = Bench.timed_fn(lambda: op.lor_vcycle(b, opk, prec=F32), 10, 2)
        row = {"lor_levels": info["rows"], "lor_nnz": info["nnz"],
               "lor_setup_ms": round(info["setup_ms"], 1), "vcycle_ms": round(ms_v, 3),
               "vcycle_fp32_ms": round(ms_v32, 3)}
        ns = opk == DIFFUSION
        row["pcg_lor"] = solve(op, b, opk, precond=PRECOND_LOR, nullspace=ns)
        row["pcg_lor_fp32_vcycle"] = solve(op, b, opk, precond=PRECOND_LOR32, nullspace=ns)
        row["pcg_jacobi"] = solve(op, b, opk, nullspace=ns)
        if ns:
            row["pcg_jacobi_fp32_ir"] = solve(op, b, opk, nullspace=ns, mode=1)
        log(f"[bench] lor {name}: levels {info['rows']}, setup {info['setup_ms']:.0f} ms, "
            f"v-cycle {ms_v:.3f} ms (FP32 {ms_v32:.3f} ms), lor {row['pcg_lor']}, "
            f"lor fp32 v-cycle {row['pcg_lor_fp32_vcycle']}, jacobi {row['pcg_jacobi']}")
        out[name] = row
        op.close()
    return out


LOR_SWEEP = [(2, 64), (3, 43), (4, 32), (5, 26), (6, 21), (7, 18), (8, 16)]


def run_lor_sweep(a):
    """The LOR preconditioner across orders (Section 7.1's question: iterations against p
    and h): the pure-Neumann Poisson problem to 1e-10 on ~2.1M-DoF meshes for p = 2..8,
    CG preconditioned by the FP32 V-cycle against Jacobi; iterations, time and the host
    set-up of the multigrid."""
    import torch
    from paper_1910_03032_amd import DIFFUSION, PRECOND_LOR32, Operator
    from workloads import BoxMesh, uniform
    rows = []
    for p, ne in LOR_SWEEP:
        m = BoxMesh(ne, p)
        op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=np_zeros(m.ndof))
        op.set_coeffs(0.0, 1.0, None)
        info = op.lor_setup(DIFFUSION)
        b = torch.as_tensor(uniform(m.ndof, seed=1), device="cuda")
        row = {"p": p, "elements": f"{ne}^3", "ndof": m.ndof, "lor_levels": info["rows"],
               "lor_setup_ms": round(info["setup_ms"], 1)}
        for name, kw in (("lor_fp32_vcycle", {"precond": PRECOND_LOR32}), ("jacobi", {})):
            op.pcg(b, op=DIFFUSION, rtol=1e-10, nullspace=True, check_every=16, maxit=20000, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, res = op.pcg(b, op=DIFFUSION, rtol=1e-10, nullspace=True, check_every=16, maxit=20000, **kw)
            torch.cuda.synchronize()
            row[name] = {"ms": round((time.perf_counter() - t) * 1e3, 2), "iters": res.iters[0],
                         "true_rel_res": res.true_rel_res[0], "status": res.status}
        log(f"[bench] lor sweep p={p} {ne}^3 ndof={m.ndof}: lor {row['lor_fp32_vcycle']}, "
            f"jacobi {row['jacobi']}, setup {row['lor_setup_ms']} ms")
        rows.append(row)
        op.close()
    return {"workload": "lor_sweep", "rows": rows}


def np_zeros(n):
    import numpy as np
    return np.zeros(n, dtype=np.uint8)


def run_sweep(a, steps=20, warmup=3):
    torch = __import__("torch")
    rows = []
    for p, ne in SWEEP:
        B = Bench(ne, p, 1e3, 1.0)
        r64 = B.apply_rate(torch.float64, steps=steps, warmup=warmup)
        r32 = B.apply_rate(torch.float32, steps=steps, warmup=warmup)
        rows.append({"p": p, "elements": f"{ne}^3", "ndof": B.m.ndof, "fp64": r64, "fp32": r32})
        log(f"[bench] sweep p={p}: fp64 {r64['GDoF/s']} GDoF/s ({r64['hbm_frac']:.3f} of HBM), "
            f"fp32 {r32['GDoF/s']} GDoF/s")
        B.close()
        del B
        torch.cuda.empty_cache()
    return {"workload": "sweep", "rows": rows}


def run_size_sweep(a):
    """Throughput of the FP64 mass (M) and diffusion (L = K(nu)) applies against problem size
    for p = 2..6, the view of the paper's operator-throughput figure (Section 6): from a
    few thousand DoFs (launch-bound, working set inside the 256 MB last-level cache) to
    1e7+ DoFs.  One operator copy, so small sizes run from that cache, as in the paper."""
    torch = __import__("torch")
    from paper_1910_03032_amd import DIFFUSION, MASS
    from workloads import normal
    rows = []
    for p in (2, 3, 4, 5, 6):
        sizes = (2, 4, 8, 16, 32, 64, 128) if p == 2 else (2, 4, 8, 16, 32, 64) if p == 3 else \
            (2, 4, 8, 16, 32, 48)
        for ne in sizes:
            B = Bench(ne, p, 1.0, 1.0)
            N = B.m.ndof
            x = torch.as_tensor(normal(N, seed=1), device=B.dev)
            y = torch.empty_like(x)
            row = {"p": p, "elements": f"{ne}^3", "ndof": N}
            for name, opk in (("M", MASS), ("L", DIFFUSION)):
                ms = B.timed(lambda: B.op.apply(x, op=opk, out=y), steps=max(a.steps, 20),
                             warmup=max(a.warmup, 3))
                row[name] = {"us": round(ms * 1e3, 2), "GDoF/s": round(N / (ms * 1e-3) / 1e9, 3)}
            rows.append(row)
            log(f"[bench] size sweep p={p} {ne}^3 ({N} DoFs): M {row['M']['GDoF/s']} GDoF/s, "
                f"L {row['L']['GDoF/s']} GDoF/s")
            B.close()
            del B, x, y
            torch.cuda.empty_cache()
    return {"workload": "size_sweep", "rows": rows}


def stokes_bytes(nelem, p, nv, npres):
    """Bytes a Stokes block apply must move: the folded Helmholtz factors (7 per point) and
    the coupling factors (9 per point) once, u and p read and y_u, y_p written once, both
    element->DoF maps once."""
    q = p + 2
    return nelem * q ** 3 * (7 + 9) * 8 + 2 * (3 * nv + npres) * 8 + nelem * ((p + 1) ** 3 + p ** 3) * 4


def run_stokes(a):
    """Taylor-Hood Stokes block operator apply (velocity Q_p, pressure Q_{p-1}) on 32^3
    hexes for p = 2..6: y_u = H u + G p, y_p = -D u with H = 1e3 M + K(nu)."""
    import torch
    from paper_1910_03032_amd import Operator
    from workloads import TaylorHoodMesh, normal, nu_c2
    rows = []
    for p in (2, 3, 4, 5, 6):
        m = TaylorHoodMesh(32, p)
        v = m.vel
        op = Operator(v.elem_xyz, v.elem_dofs, v.ndof, p, ess=v.ess)
        xq = op.qpoint_coords()
        op.set_coeffs(1e3, 1.0, nu_c2(xq[0], xq[1], xq[2]))
        op.setup_pressure(m.pres_dofs, m.npres)
        dev = torch.device("cuda", 0)
        u = torch.as_tensor(normal(3 * v.ndof, seed=1), device=dev).reshape(3, -1)
        pres = torch.as_tensor(normal(m.npres, seed=2), device=dev)
        for _ in range(a.warmup):
            op.stokes_apply(u, pres)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        for _ in range(a.steps):
            op.stokes_apply(u, pres)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        ndof = 3 * v.ndof + m.npres
        nbytes = stokes_bytes(v.nelem, p, v.ndof, m.npres)
        row = {"p": p, "elements": "32^3", "velocity_dofs": 3 * v.ndof, "pressure_dofs": m.npres,
               "us": round(ms * 1e3, 2), "GDoF/s": round(ndof / (ms * 1e-3) / 1e9, 3),
               "algorithmic_bytes": nbytes,
               "algorithmic_GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
               "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        rows.append(row)
        log(f"[bench] stokes p={p}: {row['us']} us, {row['GDoF/s']} GDoF/s, {row['hbm_frac']:.3f} of HBM")
        op.close()
        del op
        torch.cuda.empty_cache()
    return {"workload": "stokes_32e", "rows": rows}


def run_projection(a):
    """Velocity-correction projection steps (Section 4.2, BDF3/EXT3 after two start-up
    steps) on 32^3 hexes at p = 4 (3 x 2.1M velocity DoFs + 2.1M pressure DoFs), nu = 0.01,
    dt = 1e-3, no-slip walls, from a smooth velocity vanishing on the walls; solves to a
    relative residual of 1e-10.  Reports the time per step and the iterations of the
    pressure (pure-Neumann CG preconditioned by the LOR multigrid V-cycle in FP64 or FP32
    arithmetic, or by Jacobi with FP32 inner solves in FP64 refinement) and velocity (three-member Jacobi-PCG) solves."""
    from workloads import BoxMesh
    from paper_1910_03032_amd import PRECOND_JACOBI, PRECOND_LOR, PRECOND_LOR32
    ne, p = 32, 4
    m = BoxMesh(ne, p)
    rows = []
    for name, pre, mode, vmode in (("lor", PRECOND_LOR, 0, 0), ("lor_fp32_vcycle", PRECOND_LOR32, 0, 0),
                                   ("lor_fp32_vcycle_velocity_ir", PRECOND_LOR32, 0, 1),
                                   ("jacobi_fp32_ir", PRECOND_JACOBI, 1, 0)):
        rows.append(projection_row(a, m, ne, p, name, pre, mode, vmode))
    return {"workload": "projection_32e", "rows": rows}


def projection_row(a, m, ne, p, name, pressure_precond, pressure_mode, velocity_mode=0):
    import torch
    from paper_1910_03032_amd import ProjectionStepper
    t0 = time.perf_counter()
    st = ProjectionStepper(m.elem_xyz, m.elem_dofs, m.ndof, p, m.ess, dt=1e-3, nu=0.01, order=3,
                           rtol=1e-10, pressure_precond=pressure_precond, pressure_mode=pressure_mode,
                           velocity_mode=velocity_mode)
    xyz = torch.as_tensor(node_positions(m, p), device=st.device)
    bump = (xyz * (1 - xyz)).prod(dim=1) * 64.0
    u = torch.stack([bump * torch.sin(torch.pi * xyz[:, 1]), bump * torch.cos(torch.pi * xyz[:, 2]),
                     bump * torch.sin(torch.pi * xyz[:, 0])])
    u[:, torch.as_tensor(m.ess.astype(bool), device=st.device)] = 0.0
    for _ in range(max(a.warmup, 3)):
        u, _p = st.step(u)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    its_p, its_u = [], []
    steps = max(1, min(a.steps, 10))
    e0.record(stream)
    for _ in range(steps):
        u, _p = st.step(u)
        its_p.append(st.last["pressure"].iters[0])
        its_u.append(max(st.last["velocity"].iters))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    row = {"pressure_solver": name, "elements": f"{ne}^3", "p": p, "velocity_dofs": 3 * m.ndof,
           "pressure_dofs": m.ndof, "ms_per_step": round(ms, 2), "pressure_iters": its_p,
           "velocity_iters": its_u, "setup_and_warmup_s": round(setup_s, 2),
           "kinetic_energy_proxy": float((u * u).sum())}
    log(f"[bench] projection step 32^3 p=4 ({name}): {row['ms_per_step']} ms, pressure iterations "
        f"{its_p}, velocity iterations {its_u}")
    st.close()
    return row


def node_positions(m, p):
    """Physical GLL node positions of the box mesh through each element's trilinear map
    (input generation: the start field of the projection workload)."""
    import numpy as np
    t1 = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    s = (np.concatenate([[-1.0], t1, [1.0]]) + 1.0) / 2.0
    n = p + 1
    l = np.arange(n ** 3)
    a, b, c = s[l % n], s[(l // n) % n], s[l // (n * n)]
    w = np.stack([(1 - a) * (1 - b) * (1 - c), a * (1 - b) * (1 - c), (1 - a) * b * (1 - c),
                  a * b * (1 - c), (1 - a) * (1 - b) * c, a * (1 - b) * c, (1 - a) * b * c,
                  a * b * c], axis=1)  # [n^3, 8]
    x = np.zeros((m.ndof, 3))
    x[m.elem_dofs.reshape(-1)] = np.einsum("lv,evr->elr", w, m.elem_xyz).reshape(-1, 3)
    return x


def run_convection(a):
    """Convection term N(u) (three velocity components) over p = 1..8, the throughput-vs-order
    view of the nonlinear term (Section 6, figure on the shared-memory convection
    evaluation), 1.8-4.8 M DoFs per component (32^3 hexes at p = 4, 24^3 at p = 7): GDoF/s
    over the 3 N velocity DoFs; bytes = coupling factors (9 per point) once, u read and N(u)
    written once, the map once."""
    import torch
    from paper_1910_03032_amd import Operator
    from workloads import BoxMesh, normal
    rows = []
    for p, ne in ((1, 128), (2, 64), (3, 40), (4, 32), (5, 28), (6, 24), (7, 24), (8, 20)):
        m = BoxMesh(ne, p)
        op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=m.ess)
        dev = torch.device("cuda", 0)
        u = torch.as_tensor(normal(3 * m.ndof, seed=1), device=dev).reshape(3, -1)
        for _ in range(a.warmup):
            op.convection(u)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        for _ in range(a.steps):
            op.convection(u)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        q = p + 2
        nbytes = m.nelem * q ** 3 * 9 * 8 + 2 * 3 * m.ndof * 8 + m.nelem * (p + 1) ** 3 * 4
        row = {"p": p, "elements": f"{ne}^3", "velocity_dofs": 3 * m.ndof, "us": round(ms * 1e3, 2),
               "GDoF/s": round(3 * m.ndof / (ms * 1e-3) / 1e9, 3), "algorithmic_bytes": nbytes,
               "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        rows.append(row)
        log(f"[bench] convection p={p}: {row['us']} us, {row['GDoF/s']} GDoF/s, {row['hbm_frac']:.3f} of HBM")
        op.close()
        del op
        torch.cuda.empty_cache()
    return {"workload": "convection", "rows": rows}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no "
                                   "multi-GPU path (the apply would shard by element slabs with "
                                   "an interface-plane exchange, which is not built)",
                          "n_gpus": a.gpus}))
        return 2
    if a.copy_mb > 0:
        return copy_calibration(a.copy_mb)
    import torch
    from workloads import WORKLOADS
    torch.cuda.set_device(0)
    if a.workload == "sweep":
        out = run_sweep(a)
    elif a.workload == "mass_neumann":
        out = run_mass_neumann(a)
    elif a.workload == "stokes_32e":
        out = run_stokes(a)
    elif a.workload == "convection":
        out = run_convection(a)
    elif a.workload == "size_sweep":
        out = run_size_sweep(a)
    elif a.workload == "projection_32e":
        out = run_projection(a)
    elif a.workload == "lor_p4_32e":
        out = run_lor(a)
    elif a.workload == "lor_sweep":
        out = run_lor_sweep(a)
    else:
        wl = WORKLOADS[a.workload]
        if a.workload == "vector_helmholtz_p7_24e":
            out = run_vector(a, wl)
        elif a.workload == "adjoint_p5_20e":
            out = run_adjoint(a, wl)
        elif a.workload == "large_p8_40e":
            out = run_large(a, wl)
        else:
            out = run_main(a, wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
