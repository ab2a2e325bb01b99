"""ORACLE -- test infrastructure only: times the oracle on the host for the benchmark's
CPU-baseline leg (one core and every core) and counts its floating-point operations.

Run as a script in its own process (the library to load is chosen at import), printing one
JSON object: python -m oracle.cpu_bench <nx> <order> <seconds per leg>.
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import tempfile
import time


def host_info():
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "L3 cache")
        info["lscpu"] = {k.strip(): v.strip() for k, v in (ln.split(":", 1) for ln in out.splitlines() if ":" in ln)
                         if k.strip() in keep}
    except Exception as e:   # lscpu missing: record why
        info["lscpu"] = str(e)
    return info


def main():
    nx, order, budget = int(sys.argv[1]), int(sys.argv[2]), float(sys.argv[3])
    from oracle import oracle as O
    from oracle.oracle import Oracle
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1903_06304_amd import inputs as I
    case = I.config_c4(nx=nx, p=order)
    o = Oracle(case.prm, case.mesh)
    dof = 4 * case.mesh.E * case.mesh.Np
    threads = len(os.sched_getaffinity(0))
    out = {"openmp": bool(O.lib().ora_openmp()), "library": O._LIB, **host_info()}
    for leg, nt in (("one_core", 1), ("all_cores", threads)):
        o.set_threads(nt)
        o.residual(case.q)
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget or n < 2:
            o.residual(case.q)
            n += 1
        dt = time.perf_counter() - t0
        out[leg] = {"threads": nt, "evals": n, "seconds": dt, "dof_per_s": dof * n / dt}
    # exact operation count of one evaluation (the count is per element, so a small periodic
    # mesh of the same kind gives it; scaled to the workload's element count)
    small = I.config_c4(nx=8, p=order)
    os_ = Oracle(small.prm, small.mesh)
    _, cnt = os_.count_residual(small.q)
    scale = case.mesh.E / small.mesh.E
    out["flops_per_residual"] = {k: int(v * scale) for k, v in cnt.items()}
    out["flops_per_dof"] = sum(cnt.values()) / (4 * small.mesh.E * small.mesh.Np)
    print(json.dumps(out))


if __name__ == "__main__":
    if len(sys.argv) > 4 and sys.argv[4] == "--native":
        # rebuild at -O3 -march=native with OpenMP on this host and time that build
        from oracle import oracle as O
        d = tempfile.mkdtemp(prefix="oracle_native_")
        path = O.build_native(os.path.join(d, "liboracle_native.so"))
        env = dict(os.environ, LMFR_ORACLE_LIB=path)
        r = subprocess.run([sys.executable, "-m", "oracle.cpu_bench", *sys.argv[1:4]], env=env,
                           capture_output=True, text=True, cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        sys.stdout.write(r.stdout)
        sys.stderr.write(r.stderr)
        sys.exit(r.returncode)
    main()
