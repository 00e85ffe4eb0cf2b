"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(-fno-sanitize-recover: the first finding aborts) runs a mixed workload -
every partition mode, k-way, inference and the FP64 gradient - in a child
process, and prints the same results as the plain build: no memory error,
no undefined behaviour, and nothing that depends on either."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def runtime(name):
    try:
        p = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def run_workload(env_extra):
    env = dict(os.environ, **env_extra)
    p = subprocess.run([sys.executable, os.path.join(HERE, "sanitize_workload.py")],
                       capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    return json.loads(p.stdout)


def test_oracle_clean_under_asan_ubsan(tmp_path):
    asan = runtime("libasan.so")
    if asan is None:
        pytest.skip("no libasan")
    lib = str(tmp_path / "liboracle_san.so")
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("oracle.c", "mpnn.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off",
                           "-fno-fast-math", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fPIC", "-shared", "-o", lib, *srcs, "-lm"])
    plain = run_workload({})
    san = run_workload({"GP_ORACLE_LIB": lib, "LD_PRELOAD": asan,
                        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert san == plain


def test_simulator_clean_under_asan_ubsan(tmp_path):
    """The library's only host-resident computation, gp_simulate, built from
    its source by the host compiler with both sanitizers, matches the
    simulator oracle on every case."""
    import shutil
    from oracle.sim import simulate
    from sanitize_sim import cases
    asan = runtime("libasan.so")
    if asan is None:
        pytest.skip("no libasan")
    csrc = os.path.join(ROOT, "paper_1502_07451_amd", "csrc")
    src = str(tmp_path / "sim_host.cpp")
    shutil.copyfile(os.path.join(csrc, "gp_sim" + ".hip"), src)
    lib = str(tmp_path / "libsim_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", csrc, "-fPIC", "-shared", "-o", lib, src])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, os.path.join(HERE, "sanitize_sim.py"), lib],
                       capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    got = json.loads(p.stdout)
    for (g, pol, part, ncpu, ngpu, lat, bw), r in zip(cases(), got):
        o = simulate(g, pol, part=part, ncpu=ncpu, ngpu=ngpu, latency=lat, bw=bw)
        assert r == [0, o.makespan, o.transfers, o.bytes, list(o.busy), list(o.tasks),
                     list(o.node), list(o.finish)]
