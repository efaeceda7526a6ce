"""invaskit_matvec_noalloc (scratch from the library's static device array)
against invaskit_matvec (caller scratch): the same product, through the C
ABI, on two calls in a row with the second smaller, plus the size limit."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1602_01376_amd.setup import make_problem, rhs_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def bind():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_01376_amd import binding
    return binding


def _noalloc(bind, fac, xc):
    """y = (lambda I + K~) x through invaskit_matvec_noalloc; xc is the
    (r, N) contiguous tensor whose memory is the column-major N x r x."""
    r = xc.shape[0]
    yc = torch.full_like(xc, float("nan"))
    st = bind.library().invaskit_matvec_noalloc(fac.handle, C.c_void_p(xc.data_ptr()), r, fac.n,
                                                C.c_void_p(yc.data_ptr()), fac.n)
    torch.cuda.synchronize()
    return st, yc.t()


def test_noalloc_matvec_matches_matvec(bind):
    """Two calls in a row, the second on a smaller problem with fewer
    columns: each equals invaskit_matvec's product to FP64 rounding (the
    same kernels in the same order, so in practice bit for bit).  Then a
    product too large for the static array is refused before any launch,
    and the array still serves the next call."""
    cases = [(make_problem("susy", n=8192, depth=5), 3), (make_problem("tiny", n=2048, depth=3), 1)]
    facs = []
    for pb, r in cases:
        _say("noalloc matvec", pb.name, pb.n, r)
        fac = bind.Factorization(pb, pb.lam, precision="fp64")
        facs.append(fac)
        x = torch.from_numpy(rhs_for(pb, nrhs=r, seed=11))
        st, y = _noalloc(bind, fac, bind._colmajor(x))
        assert st == 0, bind.last_error(fac.handle)
        y_ref = fac.matvec(x)
        y, y_ref = y.cpu().numpy(), y_ref.cpu().numpy().reshape(y.shape)
        scale = np.abs(y_ref).max(axis=0)
        err = (np.abs(y - y_ref).max(axis=0) / scale).max()
        _say("  max column-relative difference", err)
        assert err <= 1e-14
    # 4096 columns of the 8,192-point problem need about 300 MB of scratch
    big = facs[0]
    need = C.c_size_t()
    assert bind.library().invaskit_matvec_workspace_bytes(big.handle, 4096, C.byref(need)) == 0
    assert need.value > (64 << 20)
    xc = torch.zeros((4096, big.n), dtype=torch.float64, device="cuda")
    st, _ = _noalloc(bind, big, xc)
    assert st == bind.E_WORKSPACE and "static scratch" in bind.last_error(big.handle)
    pb, r = cases[1]
    x = torch.from_numpy(rhs_for(pb, nrhs=r, seed=12))
    st, y = _noalloc(bind, facs[1], bind._colmajor(x))
    assert st == 0
    y_ref = facs[1].matvec(x).cpu().numpy().reshape(-1, r)
    assert np.abs(y.cpu().numpy() - y_ref).max() <= 1e-14 * np.abs(y_ref).max()
    for f in facs:
        f.close()
