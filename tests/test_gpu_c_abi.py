"""The C ABI driven from a C program (tests/c_abi/plain_method.c: HIP runtime
and the library only, no Python in the process): the plain-method workload
(64^3, constant 2000 m/s, centred 15 Hz Ricker, 100 steps) against the FP64
oracle, bar rel-L2 <= 1e-5 for u^100 and u^99."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from compare import check_close
import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_abi", "_build", "plain_method")


def _exe():
    if not os.path.exists(EXE):  # not built yet: build it (gcc, seconds)
        import importlib.util
        spec = importlib.util.spec_from_file_location("_c_abi_build", os.path.join(HERE, "c_abi", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    return EXE


@pytest.fixture(autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_c_program_plain_method_vs_oracle(tmp_path):
    n, nt = 64, 100
    c = workloads.config_plain(n, n, n, nt=nt)
    wav = tmp_path / "wavelet.f32"
    out = tmp_path / "u.f32"
    c["amp"].astype(np.float32).tofile(wav)
    print(f"case: C program, plain method {n}^3, {nt} steps", flush=True)
    r = subprocess.run([_exe(), str(n), str(n), str(n), str(nt), str(wav), str(out)], capture_output=True,
                       text=True, timeout=120)
    print(r.stdout.strip(), r.stderr.strip(), flush=True)
    assert r.returncode == 0, r.stderr
    u = np.fromfile(out, dtype=np.float32).reshape(2, n, n, n)
    kap = oracle.kappa(c["v"], c["dt"], c["h"])
    z = np.zeros(kap.shape)
    ref_n, ref_nm1 = oracle.leapfrog(kap, z, z, 4, nt, src_idx=c["src_idx"], amp=c["amp"])
    check_close(u[0], ref_n, 1e-5, f"u^{nt}")
    check_close(u[1], ref_nm1, 1e-5, f"u^{nt - 1}")
