"""Serving runtime through the C ABI: continuous batching of many streams of uneven widths in
grouped launches, admission by device-memory footprint, and results that are the same alone, in
a mix and through a single handle (every block is planned from its own shape, so the same bits)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import quantized_blocks, split_blocks

pytestmark = pytest.mark.gpu

L, K, B = 40, 10, 10
SPECS = [  # n, blocks (rows), data seed, Omega seed
    (777, [1, 17, 300, 513, 700], 11, 21),
    (1536, [512, 512, 512, 464], 12, 22),
    (300, [256, 256, 256, 132], 13, 23),
    (2048, [1024, 100, 900], 14, 24),
]


@pytest.fixture(scope="module")
def data():
    import torch
    out = []
    for n, blocks, dseed, oseed in SPECS:
        m = sum(blocks)
        sig = synth.noisy_spectrum(synth.exp_spectrum(min(m, n), 8.0), 1e-6, dseed)
        A, _, _, _ = synth.small_matrix(m, n, sig, dseed)
        out.append(dict(n=n, m=m, blocks=blocks, seed=oseed, A=A,
                        At=torch.from_numpy(A.astype(np.float32)).cuda()))
    return out


def _single(sk, d, mode):
    import torch
    h = sk.Sketch(d["n"], d["m"], max(d["blocks"]), K, L, B, compute=mode, seed=d["seed"])
    r0 = 0
    for c in d["blocks"]:
        h.ingest(d["At"][r0:r0 + c])
        r0 += c
    Om = h.omega().cpu().numpy()
    S, V, _, rank = h.finalize()
    torch.cuda.synchronize()
    h.close()
    return S.cpu().numpy(), V.cpu().numpy(), rank, Om


def _server(sk, mode="f32", worker=False, max_group=16, state_bytes=1 << 30):
    return sk.Server(L, max_n=4096, max_m=4096, max_block_rows=1024, state_bytes=state_bytes,
                     compute=mode, src="f32", max_group=max_group, worker=worker)


def _serve(sk, srv, ds, finalize_order=None):
    """Opens every stream, submits their blocks interleaved (one block of each stream in turn),
    drives the scheduler when it has no thread, and finalizes in the given order."""
    ids, tickets = [], []
    for d in ds:
        sid, _ = srv.open(d["n"], d["m"], K, B, d["seed"])
        ids.append(sid)
    queues = [list(split_blocks(d["At"], d["blocks"])) for d in ds]
    while any(queues):
        for i, q in enumerate(queues):
            if q:
                tickets.append(srv.submit(ids[i], q.pop(0)))
        if not srv.cfg.worker:
            srv.step()
    out = {}
    for i in (finalize_order or range(len(ds))):
        S, V, _, rank = srv.finalize(ids[i])
        out[i] = (S.cpu().numpy(), V.cpu().numpy(), rank)
    return out, tickets


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_server_equals_single_handle(gpu_lib, data, mode):
    srv = _server(gpu_lib, mode)
    res, _ = _serve(gpu_lib, srv, data)
    st = srv.stats()
    srv.close()
    assert st["max_blocks_in_group"] > 1          # blocks of different streams were grouped
    assert st["finalized"] == len(data)
    for i, d in enumerate(data):
        S1, V1, r1, _ = _single(gpu_lib, d, mode)
        S2, V2, r2 = res[i]
        assert r1 == r2
        assert np.array_equal(S1, S2)
        assert np.array_equal(V1, V2)


def test_alone_and_in_the_mix(gpu_lib, data):
    srv = _server(gpu_lib, "f32", worker=True)
    alone, _ = _serve(gpu_lib, srv, data[:1])
    srv.close()
    srv = _server(gpu_lib, "f32", worker=True, max_group=3)
    mix, _ = _serve(gpu_lib, srv, data, finalize_order=[3, 1, 0, 2])
    srv.close()
    assert np.array_equal(alone[0][0], mix[0][0])
    assert np.array_equal(alone[0][1], mix[0][1])


@pytest.mark.parametrize("mode", ["f32", "bf16", "bf16x2"])
def test_matches_reference(gpu_lib, data, mode):
    """Each stream of a mixed group against the reference on its own rounded rows and Omega'."""
    srv = _server(gpu_lib, mode)
    res, _ = _serve(gpu_lib, srv, data)
    srv.close()
    for i, d in enumerate(data):
        _, _, _, Om = _single(gpu_lib, d, mode)
        ref = oracle.single_pass_pca(quantized_blocks(d["A"], d["blocks"], mode), Om, K, B)
        S, V, rank = res[i]
        assert rank == ref.rank
        assert np.max(oracle.rel_sigma_error(S, ref.S)) < 2e-4
        assert oracle.sin_theta_max(ref.V, V) < 2e-3


def test_admission_by_footprint(gpu_lib, data):
    """A budget for two of the three streams: the third waits, is admitted when the first is
    finalized, and every result still equals the single-handle one."""
    probe = _server(gpu_lib, "f32")
    foot = [probe.stream_bytes(d["n"], d["m"], K, B) for d in data[:3]]
    probe.close()
    budget = foot[0] + foot[1] + min(foot[2], foot[0]) // 2
    assert budget < sum(foot)
    srv = _server(gpu_lib, "f32", worker=False, state_bytes=budget)
    ids, adm = [], []
    for d in data[:3]:
        sid, a = srv.open(d["n"], d["m"], K, B, d["seed"])
        ids.append(sid)
        adm.append(a)
    assert adm == [True, True, False]
    assert srv.stats()["queued"] == 1
    for i, d in enumerate(data[:3]):
        r0 = 0
        for c in d["blocks"]:
            srv.submit(ids[i], d["At"][r0:r0 + c])
            r0 += c
    with pytest.raises(gpu_lib.SketchError, match="waiting for memory"):
        srv.finalize(ids[2])
    out = {}
    out[0] = srv.finalize(ids[0])
    st = srv.stats()
    assert st["queued"] == 0 and st["active"] == 2
    out[1] = srv.finalize(ids[1])
    out[2] = srv.finalize(ids[2])
    st = srv.stats()
    srv.close()
    assert st["state_peak"] <= budget
    assert st["finalized"] == 3
    for i, d in enumerate(data[:3]):
        S1, V1, _, _ = _single(gpu_lib, d, "f32")
        assert np.array_equal(S1, out[i][0].cpu().numpy())
        assert np.array_equal(V1, out[i][1].cpu().numpy())


def test_poll_returns_every_ticket(gpu_lib, data):
    srv = _server(gpu_lib, "f32", worker=True)
    _, tickets = _serve(gpu_lib, srv, data)
    seen = {}
    for _ in range(100):
        for tk, lat in srv.poll():
            seen[tk] = lat
        if len(seen) == len(tickets):
            break
    srv.close()
    assert sorted(seen) == sorted(tickets)
    assert all(lat >= 0 for lat in seen.values())


def test_server_errors(gpu_lib, data):
    d = data[0]
    srv = _server(gpu_lib, "f32")
    with pytest.raises(gpu_lib.SketchError, match="unknown stream"):
        srv.submit(12345, d["At"][:10])
    sid, _ = srv.open(d["n"], d["m"], K, B, 1)
    with pytest.raises(gpu_lib.SketchError, match="max_block_rows"):
        srv.submit(sid, d["At"][:1025])
    srv.submit(sid, d["At"][:100])
    S, V, _, rank = srv.finalize(sid)
    assert rank == L
    with pytest.raises(gpu_lib.SketchError, match="unknown stream"):
        srv.submit(sid, d["At"][:10])
    with pytest.raises(gpu_lib.SketchError, match="exceeds the state budget"):
        big = _server(gpu_lib, "f32", state_bytes=1 << 20)
        big.open(d["n"], d["m"], K, B, 1)
    srv.close()


def _host_server(sk, mode, worker, host_slots):
    return sk.Server(L, max_n=4096, max_m=4096, max_block_rows=1024, state_bytes=1 << 30,
                     compute=mode, src="f32", max_group=16, worker=worker, host_slots=host_slots)


@pytest.mark.parametrize("mode,worker", [("f32", False), ("bf16", True), ("bf16x2", False)])
def test_pinned_host_blocks(gpu_lib, data, mode, worker):
    """Streams 0 and 2 submit pinned host rows, 1 and 3 device rows, through two staging slots
    (fewer than the host blocks of one round, so host blocks wait for a slot): the staged copy
    is the same rows, so every stream equals its single-handle result bit for bit."""
    import torch
    srv = _host_server(gpu_lib, mode, worker, host_slots=2)
    host = {0: torch.from_numpy(data[0]["A"].astype(np.float32)).pin_memory(),
            2: torch.from_numpy(data[2]["A"].astype(np.float32)).pin_memory()}
    ids = [srv.open(d["n"], d["m"], K, B, d["seed"])[0] for d in data]
    queues = []
    for i, d in enumerate(data):
        src = host[i] if i in host else d["At"]
        queues.append(list(split_blocks(src, d["blocks"])))
    while any(queues):
        for i, q in enumerate(queues):
            if q:
                srv.submit(ids[i], q.pop(0))
        if not worker:
            srv.step()
    res = {i: srv.finalize(ids[i]) for i in range(len(data))}
    st = srv.stats()
    srv.close()
    assert st["finalized"] == len(data)
    for i, d in enumerate(data):
        S1, V1, r1, _ = _single(gpu_lib, d, mode)
        S2, V2, _, r2 = res[i]
        assert r1 == r2
        assert np.array_equal(S1, S2.cpu().numpy())
        assert np.array_equal(V1, V2.cpu().numpy())


def test_pinned_host_padded_rows(gpu_lib, data):
    """Host rows with a leading dimension above n (a column slice of a wider pinned matrix)."""
    import torch
    d = data[1]
    wide = torch.zeros(d["m"], d["n"] + 37, dtype=torch.float32).pin_memory()
    wide[:, 5:5 + d["n"]] = torch.from_numpy(d["A"].astype(np.float32))
    srv = _host_server(gpu_lib, "f32", False, host_slots=1)
    sid, _ = srv.open(d["n"], d["m"], K, B, d["seed"])
    r0 = 0
    for c in d["blocks"]:
        srv.submit(sid, wide[r0:r0 + c, 5:5 + d["n"]])
        srv.step()
        r0 += c
    S, V, _, _ = srv.finalize(sid)
    srv.close()
    S1, V1, _, _ = _single(gpu_lib, d, "f32")
    assert np.array_equal(S1, S.cpu().numpy()) and np.array_equal(V1, V.cpu().numpy())


def test_arrival_time_latency(gpu_lib, data):
    """A block stamped as arrived 0.25 s before its submit reports at least 0.25 s of latency;
    blocks stamped at submit report less than that on an idle server."""
    import time
    d = data[2]
    srv = _host_server(gpu_lib, "f32", True, host_slots=1)
    sid, _ = srv.open(d["n"], d["m"], K, B, d["seed"])
    blocks = list(split_blocks(d["At"], d["blocks"]))
    late = srv.submit(sid, blocks[0], arrival_s=srv.clock() - 0.25)
    seen = {}
    t_end = time.time() + 10
    while late not in seen and time.time() < t_end:
        seen.update(dict(srv.poll()))
    fresh = [srv.submit(sid, b) for b in blocks[1:]]
    srv.finalize(sid)
    for _ in range(10):
        seen.update(dict(srv.poll()))
    srv.close()
    assert seen[late] >= 0.25
    assert all(0 <= seen[t] < 0.25 for t in fresh)


def test_host_submit_errors(gpu_lib, data):
    import torch
    d = data[0]
    rows = torch.from_numpy(d["A"][:100].astype(np.float32))
    srv = _server(gpu_lib, "f32")                 # no staging slots
    sid, _ = srv.open(d["n"], d["m"], K, B, 1)
    with pytest.raises(gpu_lib.SketchError, match="no host staging slots"):
        srv.submit(sid, rows.pin_memory())
    srv.close()
    srv = _host_server(gpu_lib, "f32", False, host_slots=1)
    sid, _ = srv.open(d["n"], d["m"], K, B, 1)
    with pytest.raises(gpu_lib.SketchError, match="pinned"):
        srv.submit(sid, rows)                      # pageable
    with pytest.raises(ValueError, match="float32"):
        srv.submit(sid, d["At"][:10].double())
    srv.submit(sid, rows.pin_memory())
    _, _, _, rank = srv.finalize(sid)
    srv.close()
    assert rank == L
