"""Separate contexts are independent: two host threads, each with its own
context, stream and fields, step at the same time (the library's calls
release the interpreter lock, so the launches interleave); each thread's
result equals its run alone bit for bit, and an error in one thread is
reported in that thread's context only."""
import sys
import threading

import numpy as np
import pytest
import torch

import paper_1310_8232_amd as p
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def test_two_threads_two_contexts():
    shapes = [(72, 45, 37), (64, 48, 40)]
    nt = 40
    jobs = []
    for i, (nx, ny, nz) in enumerate(shapes):
        v = workloads.layered_model(nx, ny, nz, seed=500 + i)
        dt, vmax = workloads.dt_for_courant(v, 10.0)
        prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
        idx = cuda(np.array([workloads.centre_index(nx, ny, nz)], np.int64), torch.int64)
        src = p.make_src(idx, cuda(workloads.ricker(nt, dt, 25.0).reshape(-1, 1)))
        u0 = cuda(workloads.random_field(nx, ny, nz, 510 + i))
        um1 = cuda(workloads.random_field(nx, ny, nz, 520 + i))
        ra, rb = prop.run(u0.clone(), um1.clone(), nt, src)
        torch.cuda.synchronize()
        jobs.append(dict(prop=prop, src=src, u0=u0, um1=um1, ref=(ra.clone(), rb.clone())))
    print(f"case: two threads, two contexts, {nt} steps each, own streams", flush=True)
    results, errors = [None, None], []

    def work(k):
        try:
            j = jobs[k]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                a, b = j["u0"].clone(), j["um1"].clone()
                for rep in range(3):
                    a, b = j["u0"].clone(), j["um1"].clone()
                    a, b = j["prop"].run(a, b, nt, j["src"], stream=s)
                # A failing call in this thread: its message stays with this context.
                try:
                    j["prop"].step(a, a, 0, None, stream=s)
                except p.StencilError as e:
                    assert e.status == p.EALIAS
                s.synchronize()
                results[k] = (a, b, p.stencil_last_error(j["prop"].ctx))
        except Exception as e:  # reported to the main thread
            errors.append(repr(e))

    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for j, r in zip(jobs, results):
        assert r is not None
        assert torch.equal(r[0], j["ref"][0]) and torch.equal(r[1], j["ref"][1])
        assert "overlap" in r[2]
