"""The field read-out that allocates no device memory
(psmdem_read_fields_noalloc) against the allocating one (psmdem_read_fields),
through the C ABI: bit for bit on two calls in a row, the first on a lattice
of more than one staging chunk (2^20 cells) after an odd number of steps (the
in-place storage read across the AA pattern, walls with moving-wall terms,
FP32 storage, particles), the second on a smaller lattice (BF16 storage,
Kolmogorov forcing, even step).  Both also agree with the moments of the
decoded populations."""
import numpy as np
import pytest

from paper_2512_04997_amd import workloads as W

pytestmark = pytest.mark.gpu

CX = np.array([0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0], dtype=np.float64)
CY = np.array([0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1], dtype=np.float64)
CZ = np.array([0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1], dtype=np.float64)


@pytest.fixture(scope="module")
def ps():
    from paper_2512_04997_amd import psmdem
    psmdem.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return psmdem


def _check(D, force):
    rho_a, u_a = D.fields()
    rho_b, u_b = D.fields(noalloc=True)
    assert np.array_equal(rho_a, rho_b) and np.array_equal(u_a, u_b)
    f = D.populations()
    rho = f.sum(axis=0)
    mom = np.stack([CX @ f, CY @ f, CZ @ f], axis=1) + 0.5 * force
    assert np.max(np.abs(rho_b - rho)) < 1e-13
    assert np.max(np.abs(u_b - mom / rho[:, None])) < 1e-13
    assert np.max(np.abs(u_b)) > 1e-6
    return rho_b, u_b


def test_noalloc_fields_equal_the_allocating_read_out_on_two_calls(ps):
    # call 1: 128 x 128 x 72 = 1,179,648 cells (two staging chunks), odd step
    box = (128, 128, 72)
    wu = [[0.0] * 3 for _ in range(6)]
    wu[4] = [-0.02, 0.0, 0.0]
    wu[5] = [0.02, 0.0, 0.0]
    cfg = W.base_config(box, 0.7, bc=["periodic"] * 4 + ["moving"] * 2, wall_u=wu, precision="fp32")
    rng = W.SplitMix64(21)
    pos = W.rsa_spheres(rng, 20, np.full(20, 4.0), box, [True, True, False])
    D = ps.Domain(cfg, W.spheres(pos, 4.0, 1.5))
    D.step(5)
    _check(D, np.zeros(3))
    D.close()
    # call 2: a smaller lattice, BF16 storage, Kolmogorov forcing, even step
    cfg2 = W.base_config((24, 20, 16), 0.6, precision="bf16", kolm_amp=1e-3, kolm_axis=1, kolm_dir=0)
    D2 = ps.Domain(cfg2, None)
    D2.step(6)
    y = (np.arange(24 * 20 * 16) // 24) % 20
    force = np.zeros((24 * 20 * 16, 3))
    force[:, 0] = 1e-3 * np.sin(2 * np.pi * (y + 0.5) / 20)
    _check(D2, force)
    D2.close()
