"""16-bit wavefield storage (FP16, BF16) with FP32 arithmetic.

* Conversions are bit-exact round-to-nearest-even of scale * u (FP16 against
  numpy's IEEE conversion, BF16 against the bit-level definition).
* Every 16-bit tile shape and the plain kernel give identical bits.
* Error against the FP64 oracle (128^3 layered, 100 steps) stays within a
  bound derived from the storage unit roundoff (u = 2^-11 for FP16, 2^-8 for
  BF16): one rounding per stored value per step, accumulating like a random
  walk over the steps, ~sqrt(n) u ~ 5e-3 (FP16) / 4e-2 (BF16) at n = 100;
  the bounds below allow about 2x that.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from compare import check_close
import paper_1310_8232_amd as p
import workloads

pytestmark = pytest.mark.gpu
SCALE = 2.0 ** 12
BOUND_100 = {"f16": 1e-2, "bf16": 8e-2}


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def bf16_rne_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of FP32 to BF16, as the upper 16 bits (finite values)."""
    b = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_conversion_bit_exact(storage):
    nx, ny, nz = 40, 36, 30
    v = workloads.layered_model(nx, ny, nz, seed=3)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, storage=storage, storage_scale=SCALE)
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((nz, ny, nx)) * np.exp(rng.uniform(-12, 2, (nz, ny, nx)))).astype(np.float32)
    st = prop.to_storage(cuda(x))
    bits = st.view(torch.int16).cpu().numpy().view(np.uint16)
    if storage == "f16":
        ref = (x.astype(np.float32) * np.float32(SCALE)).astype(np.float16).view(np.uint16)
    else:
        ref = bf16_rne_bits(x * np.float32(SCALE))
    assert np.array_equal(bits, ref)
    back = prop.to_f32(st).cpu().numpy()
    if storage == "f16":
        ref_back = ref.view(np.float16).astype(np.float32) / np.float32(SCALE)
    else:
        ref_back = (ref.astype(np.uint32) << 16).view(np.float32) / np.float32(SCALE)
    assert np.array_equal(back, ref_back)


def _random_state(prop, shape, seed):
    nz, ny, nx = shape
    u0 = workloads.random_field(nx, ny, nz, seed + 1)
    um1 = workloads.random_field(nx, ny, nz, seed + 2)
    return prop.to_storage(cuda(u0)), prop.to_storage(cuda(um1))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("R,shape", [(4, (72, 45, 37)), (5, (72, 45, 37)), (4, (61, 29, 23)), (4, (76, 33, 21))])
def test_16bit_tiles_bit_identical(storage, R, shape):
    nx, ny, nz = shape
    v = workloads.layered_model(nx, ny, nz, seed=11)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    log(f"case: {storage} R={R} {shape}, every 16-bit tile")
    tiles = []
    # Every vector width that divides nx: 8 (16-byte accesses), 4 and 1 points.
    lists = [t for w, flag in ((8, 8), (4, 1), (1, 0)) if nx % w == 0 for t in p.stencil_list_tiles(R, flag, storage)]
    for t in lists:
        for dz in (1, 7, nz):
            for xcd in (1, 0):
                tiles.append(p.make_tile(p.TILE_ZMARCH, t.bx, t.by, t.ry, dz, t.vw, xcd, t.pf))
    tiles.append(p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1))
    assert len(tiles) > 3
    base = None
    for t in tiles:
        prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax, storage=storage, storage_scale=SCALE, tile=t)
        a, b = _random_state(prop, (nz, ny, nx), 31)
        a, b = prop.run(a, b, 6)
        torch.cuda.synchronize()
        got = (a.view(torch.int16).cpu().numpy(), b.view(torch.int16).cpu().numpy())
        if base is None:
            base = got
        else:
            assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1]), f"tile {t}"


def _error_vs_oracle(storage, n, nt):
    c = workloads.config_layered(n, n, n, nt=nt)
    prop = p.Propagator(cuda(c["v"]), c["h"], c["dt"], 4, vmax=c["vmax"], storage=storage,
                        storage_scale=SCALE if storage != "f32" else 1.0)
    src = p.make_src(cuda(c["src_idx"], torch.int64), cuda(c["amp"].reshape(-1, 1)))
    a, b = prop.run(prop.zeros(), prop.zeros(), nt, src)
    un = prop.to_f32(a).cpu().numpy() if storage != "f32" else a.cpu().numpy()
    unm1 = prop.to_f32(b).cpu().numpy() if storage != "f32" else b.cpu().numpy()
    kap = oracle.kappa(c["v"], c["dt"], c["h"])
    z = np.zeros(kap.shape)
    ref_n, ref_nm1 = oracle.leapfrog(kap, z, z, 4, nt, src_idx=c["src_idx"], amp=c["amp"])
    return (un, unm1), (ref_n, ref_nm1)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_error_vs_oracle_128_100_steps(storage):
    (un, unm1), (ref_n, ref_nm1) = _error_vs_oracle(storage, 128, 100)
    log(f"  {storage} 128^3 100 steps:")
    check_close(un, ref_n, BOUND_100[storage], "u^n")
    check_close(unm1, ref_nm1, BOUND_100[storage], "u^n-1")


@pytest.mark.slow
def test_error_vs_oracle_128_1000_steps_all_storages():
    out = {}
    for storage in ("f32", "f16", "bf16"):
        (un, unm1), (ref_n, ref_nm1) = _error_vs_oracle(storage, 128, 1000)
        out[storage] = (oracle.rel_l2(un, ref_n), oracle.rel_l2(unm1, ref_nm1))
        log(f"  {storage} 128^3 1000 steps: rel_l2 u^n {out[storage][0]:.3e}, u^n-1 {out[storage][1]:.3e}")
    assert out["f32"][0] <= 2e-4
    assert out["f16"][0] <= 1e-1 and out["bf16"][0] <= 0.5
