"""GPU parity of the in-plane (P-SV) plain form against the exact oracle.

Straight fault, alpha = 1, beta = alpha / sqrt(3), alpha dt / dx = 1/2 (the
paper's in-plane medium, App. A; with these units the P fronts sit exactly
on element ends at the collocation times, in floating point too, and the S
fronts never do); two components per element (shear slip rate ->
shear traction, opening rate -> normal traction).  Tier-A (the exact
convolution with the oracle's closed-form kernel); tolerances as for the
anti-plane dense form: relative L2 <= 1e-12, max |dT| <= 1e-11 max |T|.
"""
import math

import numpy as np
import pytest

from oracle.dense import convolve_dense
from oracle.inplane2d import InplaneProblem
from synth import smooth_slip_rate, straight_fault, uniform_slip_rate

pytestmark = pytest.mark.gpu

ALPHA, BETA, DT = 1.0, 1.0 / math.sqrt(3.0), 0.5


def _gpu(N, M, D2, graph=False):
    import torch

    from paper_1903_02118_amd.binding import BIE_MODE_INPLANE, Operator

    xa, xb = straight_fault(N)
    op = Operator.build_kernel(xa, xb, M, mode=BIE_MODE_INPLANE, alpha=ALPHA, beta=BETA, dt=DT)
    Dd = torch.from_numpy(np.ascontiguousarray(D2.reshape(D2.shape[0], -1))).to("cuda")
    Td = torch.zeros_like(Dd)
    s = torch.cuda.current_stream()
    op.reset(stream=s)
    (op.run_graph if graph else op.run)(Dd, Td, stream=s)
    torch.cuda.synchronize()
    st = op.stats()
    op.close()
    return Td.cpu().numpy().reshape(D2.shape), st


def _oracle(N, M, D2):
    xa, xb = straight_fault(N)
    pr = InplaneProblem(xa[:, 0], xb[:, 0], dt=DT, alpha=ALPHA, beta=BETA)
    Ks, Kn = pr.kernel_tensor(M)
    return np.stack([convolve_dense(Ks, D2[:, :, 0]), convolve_dense(Kn, D2[:, :, 1])], axis=2)


def _check(T, Tr):
    err = np.linalg.norm(T - Tr) / np.linalg.norm(Tr)
    assert err <= 1e-12, err
    assert np.abs(T - Tr).max() <= 1e-11 * np.abs(Tr).max()
    return err


@pytest.mark.parametrize("N,M", [(96, 120), (33, 7), (1, 1), (2, 5)])
def test_inplane_dense_matches_exact_oracle(gpu_lib, N, M):
    if N * M >= 16:
        D2 = np.stack([smooth_slip_rate(N, M, 10, 20, 31), smooth_slip_rate(N, M, 10, 20, 32)], axis=2)
    else:  # too small for a standardized field
        D2 = np.stack([uniform_slip_rate(N, M, 31), uniform_slip_rate(N, M, 32)], axis=2)
    print(f"inplane dense N={N} M={M}", flush=True)
    T, st = _gpu(N, M, D2)
    assert st["n_elem"] == N
    err = _check(T, _oracle(N, M, D2))
    print("inplane dense rel err", err, flush=True)


def test_inplane_impulse_response_is_the_kernel(gpu_lib):
    N, M = 40, 30
    j0 = 17
    D2 = np.zeros((M, N, 2))
    D2[0, j0, 0] = 1.0
    D2[0, j0 + 3, 1] = 1.0
    T, _ = _gpu(N, M, D2)
    xa, xb = straight_fault(N)
    pr = InplaneProblem(xa[:, 0], xb[:, 0], dt=DT, alpha=ALPHA, beta=BETA)
    Ks, Kn = pr.kernel_tensor(M)
    assert np.allclose(T[:, :, 0], Ks[:, :, j0], rtol=0, atol=1e-14)
    assert np.allclose(T[:, :, 1], Kn[:, :, j0 + 3], rtol=0, atol=1e-14)


def test_inplane_graph_launches_equal_eager(gpu_lib):
    N, M = 64, 50
    D2 = np.stack([smooth_slip_rate(N, M, 10, 20, 33), smooth_slip_rate(N, M, 10, 20, 34)], axis=2)
    Te, _ = _gpu(N, M, D2)
    Tg, _ = _gpu(N, M, D2, graph=True)
    assert np.array_equal(Te, Tg)
