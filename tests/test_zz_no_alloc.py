"""The no-allocation product (dda_apply_noalloc) against dda_apply through the
C ABI: bitwise equal (the same kernels), on two calls in a row, the second
with a smaller input, in FP64 and with the FP32 matvec; and its errors (an
input beyond its fixed work memory, a tensor FFT not yet built)."""
import numpy as np
import pytest
import torch

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dda():
    import paper_1202_3424_amd as pkg
    assert torch.cuda.is_available()
    return pkg


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _oblique():
    kh = np.array([[1, 0, 0], [0.36, 0.48, 0.8], [0.0, 0.6, 0.8]])
    e0 = np.array([[0, 1, 0], np.array([0.8, -0.6, 0]) + 1j * np.cross([0.36, 0.48, 0.8], [0.8, -0.6, 0]),
                   [1, 0, 0]])
    return kh, e0


@pytest.mark.parametrize("precision", ["fp64", "fp32_matvec"])
def test_noalloc_apply_matches_apply_twice(dda, precision):
    kh, e0 = _oblique()
    d = w.workload("ellipsoid51k")
    big = dda.Target(d["ijk"], d["m"])
    rng = np.random.default_rng(3)
    pts = np.unique(rng.integers(0, [21, 17, 30], size=(900, 3)), axis=0).astype(np.int32)
    small = dda.Target(pts, np.where(np.arange(len(pts)) % 4 == 0, 1.5 + 0.2j, 2.0 + 0.1j))
    opts = dda.Options.for_size_parameter(4.0, precision=precision)
    # first call: the 51,488-site ellipsoid with three right-hand sides;
    # second: a smaller ragged two-material target with two
    for tgt, nq, seed in ((big, 3, 31), (small, 2, 32)):
        x = _cuda(w.random_vectors(seed, (nq, tgt.n_sites, 3)))
        ref = dda.apply(tgt, opts, kh[:nq], e0[:nq], x)      # builds the tensor FFT
        y = torch.full_like(x, complex(np.nan, np.nan))
        dda.apply_noalloc(tgt, opts, kh[:nq], e0[:nq], x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (tgt.n_sites, nq, precision)


def test_noalloc_apply_errors(dda):
    from paper_1202_3424_amd import DDAError
    kh, e0 = _oblique()
    pts = w.sphere_integer(5.0)
    tgt = dda.Target(pts, 1.33 + 0.01j)
    x = _cuda(w.random_vectors(33, (1, tgt.n_sites, 3)))
    y = torch.empty_like(x)
    opts = dda.Options.for_size_parameter(2.0)
    with pytest.raises(DDAError) as e:          # tensor FFT not built for this kd yet
        dda.apply_noalloc(tgt, opts, kh[:1], e0[:1], x, y)
    assert e.value.status == 1 and "not built" in str(e.value)
    dda.apply(tgt, opts, kh[:1], e0[:1], x)
    dda.apply_noalloc(tgt, opts, kh[:1], e0[:1], x, y)
    with pytest.raises(DDAError):               # another kd: not built either
        dda.apply_noalloc(tgt, dda.Options.for_size_parameter(2.5), kh[:1], e0[:1], x, y)
    # a 96^3 brick in FP64: 192^3 grid, 3 x 16 bytes per point = 340 MB > 128 MiB
    big = dda.Target(w.brick(96, 96, 96), 1.33 + 0.01j)
    xb = torch.zeros((1, big.n_sites, 3), dtype=torch.complex128, device="cuda")
    yb = torch.empty_like(xb)
    dda.apply(big, opts, kh[:1], e0[:1], xb)
    with pytest.raises(DDAError) as e:
        dda.apply_noalloc(big, opts, kh[:1], e0[:1], xb, yb)
    assert e.value.status == 1 and "work memory" in str(e.value)
