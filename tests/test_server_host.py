"""Host-only checks of the serving ABI: workspace and per-stream sizes (the admission charge) and
configuration validation, without touching a GPU."""
import pytest

import paper_1704_07669_amd as sk


def _srv(**kw):
    base = dict(compute=sk.F32, src=sk.F32, l=40, max_group=16, max_n=32768, max_m=200000,
                max_block_rows=4096, state_bytes=4 << 30, worker=1, host_slots=0)
    base.update(kw)
    return sk.sketch_server_config(**base)


def _stream(**kw):
    base = dict(n=20000, m_capacity=100000, max_block_rows=4096, k=20, l=40, b=10, compute=sk.F32,
                host_slots=0, host_src=sk.F32, want_u=0, omega_from_seed=1, seed=3)
    base.update(kw)
    return sk.sketch_config(**base)


def _align(x):
    return (x + 255) // 256 * 256


@pytest.mark.parametrize("compute,op,acc", [(sk.F32, 4, 4), (sk.BF16, 2, 4), (sk.F64, 8, 8)])
def test_stream_bytes_is_the_resident_state(compute, op, acc):
    """Omega (FP64 + operand copy), G (m x l_p), H (n x l_p FP64) and the control block."""
    src = sk.F64 if compute == sk.F64 else sk.F32
    scfg = _srv(compute=compute, src=src)
    n, m = 20000, 100000
    LP = 48
    NP = (n + 511) // 512 * 512
    MC = (m + 63) // 64 * 64
    want = (_align(NP * LP * 8) + _align(NP * LP * op) + _align(MC * LP * acc) +
            _align(NP * LP * 8) + 256)
    assert sk.sketch_server_stream_bytes(scfg, _stream(compute=compute, host_src=src)) == want


def test_workspace_grows_with_budget_and_group():
    a = sk.sketch_server_workspace_size(_srv())
    b = sk.sketch_server_workspace_size(_srv(state_bytes=(4 << 30) + (1 << 20)))
    c = sk.sketch_server_workspace_size(_srv(max_group=32))
    assert b - a == 1 << 20
    assert c > a


def test_workspace_holds_the_staging_slots():
    """Each pinned-host staging slot holds max_block_rows rows of max_n source elements, the
    rows padded to 64 elements."""
    a = sk.sketch_server_workspace_size(_srv())
    for slots in (1, 3):
        b = sk.sketch_server_workspace_size(_srv(host_slots=slots))
        assert b - a == slots * _align(4096 * 32768 * 4)
    a = sk.sketch_server_workspace_size(_srv(max_n=1000, src=sk.BF16, compute=sk.BF16))
    b = sk.sketch_server_workspace_size(_srv(max_n=1000, src=sk.BF16, compute=sk.BF16,
                                             host_slots=2))
    assert b - a == 2 * _align(4096 * 1024 * 2)


@pytest.mark.parametrize("bad,msg", [
    (dict(compute=sk.FP8_E4M3), "compute"),
    (dict(src=sk.BF16), "src"),
    (dict(l=0), "l must"),
    (dict(max_group=0), "max_group"),
    (dict(max_n=10), "max_n"),
    (dict(worker=2), "worker"),
    (dict(host_slots=-1), "host_slots"),
    (dict(host_slots=65), "host_slots"),
])
def test_server_config_rejected(bad, msg):
    with pytest.raises(sk.SketchError, match=msg):
        sk.sketch_server_workspace_size(_srv(**bad))


@pytest.mark.parametrize("bad,msg", [
    (dict(n=40000), "n must"),
    (dict(l=20, k=10), "l must equal"),
    (dict(compute=sk.BF16), "compute must equal"),
    (dict(m_capacity=300000), "m_capacity"),
    (dict(max_block_rows=8192), "max_block_rows"),
    (dict(omega_from_seed=0), "seed"),
    (dict(host_slots=2), "device rows"),
    (dict(b=7), "b must"),
])
def test_stream_config_rejected(bad, msg):
    with pytest.raises(sk.SketchError, match=msg):
        sk.sketch_server_stream_bytes(_srv(), _stream(**bad))
