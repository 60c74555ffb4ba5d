"""bdu_update_noalloc (the update for callers that cannot allocate) gives
the same factors as bdu_update, bit for bit, through the C ABI: two calls in
a row, the second on a smaller problem than the first (the shared device
scratch keeps the first call's contents), host and device inputs, and the
size limit."""
import numpy as np
import pytest

from paper_2509_02840_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bdu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_02840_amd import bdu as B
    B.lib()
    return B


def _eq(name, x, y):
    x, y = np.asarray(x), np.asarray(y)
    assert x.shape == y.shape, name
    bad = np.flatnonzero(~(x == y).ravel())
    assert bad.size == 0, f"{name}: {bad.size} of {x.size} differ, first at {bad[0]}"


def _twins(bdu, m, n, seed):
    f = W.factorization(m, n, seed)
    return f, bdu.Handle(f.Q, f.d, f.e, f.P), bdu.Handle(f.Q, f.d, f.e, f.P)


@pytest.mark.parametrize("device_inputs", [False, True])
def test_noalloc_equals_update_on_two_calls(bdu, oracle, device_inputs):
    import torch
    for m, n, r, seed in [(300, 200, 3, 1), (70, 53, 2, 2)]:  # the second call is smaller
        f, h1, h2 = _twins(bdu, m, n, seed)
        (B, C), = W.gaussian_updates(m, n, 1, seed + 10, r=r)
        h1.update(B, C)
        if device_inputs:
            Bt = torch.from_numpy(B.T.copy()).to("cuda:0").T
            Ct = torch.from_numpy(C.T.copy()).to("cuda:0").T
            h2.update_noalloc(Bt, Ct)
        else:
            h2.update_noalloc(B, C)
        got, want = h2.read(), h1.read()
        for nm, x, y in zip("QdeP", got, want):
            _eq(f"{m}x{n} r={r} {nm}", x, y)
        st = oracle.State(f.Q, f.d, f.e, f.P)
        oracle.bgu_update(st, B, C)
        _eq(f"{m}x{n} d vs oracle", got[1], st.d)
        _eq(f"{m}x{n} e vs oracle", got[2], st.e)
        h1.close()
        h2.close()


def test_noalloc_rejects_updates_beyond_its_scratch(bdu):
    cap = bdu.lib().bdu_noalloc_capacity()
    m, n = 2048, 2048
    r = cap // (m + n) + 1
    f = W.factorization(m, n, 5)
    h = bdu.Handle(f.Q, f.d, f.e, f.P)
    B = np.zeros((m, r), order="F")
    C = np.zeros((n, r), order="F")
    with pytest.raises(bdu.BduError) as ei:
        h.update_noalloc(B, C)
    assert ei.value.status == bdu.BDU_ESCRATCH
    for nm, x, y in zip("QdeP", h.read(), (f.Q, f.d, f.e, f.P)):
        _eq(f"unchanged {nm}", x, y)
    h.close()
