"""The QR entry point that allocates nothing (cpqr_qr_noalloc) against the
allocating cpqr_qr, through the C ABI: the same kernels run on the same data,
so Q and R must agree bit for bit.  Two calls in a row, the second with a
smaller input, check that the shared scratch array carries nothing from one
call into the next.  Sizes beyond the fixed scratch are refused on the host
before any device work."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2503_18759_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load_library()
    return P


def _colmajor(A):
    import torch
    M, R = A.shape
    return torch.from_numpy(np.asfortranarray(A).ravel(order="F")).cuda().reshape(R, M).t()


def _outputs(M, R):
    import torch
    Q = torch.full((R, M), float("nan"), dtype=torch.float64, device="cuda").t()
    Rm = torch.full((R, R), float("nan"), dtype=torch.float64, device="cuda").t()
    return Q, Rm


def _check_pair(P, M, R, seed):
    import torch
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, R))
    A[:, 1] += 3 * A[:, 0]
    a = _colmajor(A)
    Qn, Rn = _outputs(M, R)
    st = P.qr_noalloc(a, Qn, Rn)
    assert st == 0, P.noalloc_last_error()
    torch.cuda.synchronize()
    Qa, Ra = P.qr(a)
    torch.cuda.synchronize()
    assert torch.equal(Qn, Qa) and torch.equal(Rn, Ra), (M, R)
    # and the QR itself is right (the oracle's Householder QR)
    Qo, Ro = O.householder_qr(A)
    assert np.max(np.abs(Rn.cpu().numpy() - Ro)) <= 1e-12 * np.max(np.abs(Ro))
    assert np.max(np.abs(Qn.cpu().numpy() - Qo)) <= 1e-11


@pytest.mark.parametrize("big,small", [((8192, 32), (1000, 32)), ((29696, 16), (300, 16)),
                                       ((5000, 20), (40, 3))])
def test_noalloc_qr_equals_allocating_qr_twice(P, big, small):
    _check_pair(P, *big, seed=big[0] + big[1])
    _check_pair(P, *small, seed=small[0] + small[1])


def test_noalloc_qr_on_a_side_stream(P):
    import torch
    M, R = 2048, 24
    rng = np.random.default_rng(11)
    A = rng.standard_normal((M, R))
    a = _colmajor(A)
    Qn, Rn = _outputs(M, R)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        assert P.qr_noalloc(a, Qn, Rn, stream=s) == 0
    s.synchronize()
    Qa, Ra = P.qr(a)
    torch.cuda.synchronize()
    assert torch.equal(Qn, Qa) and torch.equal(Rn, Ra)


@pytest.mark.parametrize("M,R", [(8193, 32), (29697, 16), (59905, 8)])
def test_noalloc_qr_refuses_sizes_beyond_its_scratch(P, M, R):
    import torch
    a = torch.zeros((R, M), dtype=torch.float64, device="cuda").t()
    Qn, Rn = _outputs(M, R)
    assert P.qr_noalloc(a, Qn, Rn) == -2      # CPQR_EUNSUPPORTED
    msg = P.noalloc_last_error()
    assert ("scratch" in msg) or ("too large" in msg), msg
    torch.cuda.synchronize()
    assert torch.isnan(Qn).all() and torch.isnan(Rn).all()     # nothing was launched
