"""GPU: the allocation-free batched Cholesky (geneo_potrf_batched_noalloc)
against geneo_potrf_batched on the same inputs: bitwise equal factors on two
calls in a row, the second with a smaller batch, in FP64 and FP32; a batch
beyond the scratch limit is refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    from paper_2311_18783_amd import geneo
    assert torch.cuda.is_available()
    ctx = geneo.Context(0)
    yield geneo, ctx
    ctx.close()


def _batch(sizes, dt, seed):
    rng = np.random.default_rng(seed)
    lds = [((n + 127) // 128) * 128 for n in sizes]
    offs = np.cumsum([0] + [l * l for l in lds])
    buf = np.zeros(offs[-1], dtype=dt)
    for n, ld, o in zip(sizes, lds, offs):
        M = rng.standard_normal((n, n))
        full = np.eye(ld)
        full[:n, :n] = M @ M.T / n + 0.1 * np.eye(n)
        buf[o:o + ld * ld] = full.T.ravel()
    return buf, offs[:-1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_potrf_matches_allocating_entry(g, prec):
    import torch
    geneo, ctx = g
    p = geneo.FP64 if prec == "fp64" else geneo.FP32_REFINE1
    dt = np.float64 if prec == "fp64" else np.float32
    # second call smaller: fewer, smaller matrices (the scratch keeps the first call's contents)
    for call, sizes in enumerate([[1500, 700, 129, 1, 2049, 300], [640, 5, 128]]):
        buf, offs = _batch(sizes, dt, 10 + call)
        print("noalloc potrf", prec, "call", call, sizes, flush=True)
        a = torch.as_tensor(buf, device="cuda:0")
        b = a.clone()
        ctx.potrf_batched(a, sizes, offs, p)
        ctx.potrf_batched(b, sizes, offs, p, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (prec, call)
        # and the result is a Cholesky factor
        out = b.cpu().numpy()
        ld0 = ((sizes[0] + 127) // 128) * 128
        L = np.tril(out[:ld0 * ld0].reshape(ld0, ld0).T)[:sizes[0], :sizes[0]].astype(np.float64)
        A0 = buf[:ld0 * ld0].reshape(ld0, ld0).T[:sizes[0], :sizes[0]].astype(np.float64)
        u = np.finfo(dt).eps / 2
        assert np.linalg.norm(L @ L.T - A0) <= 2 * sizes[0] * u * np.linalg.norm(A0)


def test_noalloc_potrf_rejects_batches_beyond_its_scratch(g):
    import torch
    geneo, ctx = g
    # 40 matrices of ld 1024 need 40 * 2 * 1024 * 128 * 8 B = 80 MiB of FP64 inverses (> 64 MiB)
    sizes = [1024] * 40
    A = torch.zeros(1024 * 1024 * 40, dtype=torch.float64, device="cuda:0")
    offs = np.arange(40, dtype=np.int64) * 1024 * 1024
    with pytest.raises(geneo.GeneoError) as ei:
        ctx.potrf_batched(A, sizes, offs, geneo.FP64, noalloc=True)
    assert ei.value.status == "EINVAL" and "too large" in str(ei.value)
    assert not A.any()
