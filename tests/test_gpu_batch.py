"""GPU parity of fglt_batch (many small graphs, one launch) against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests._util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fg():
    import paper_2007_11111_amd as fg
    assert torch.cuda.is_available()
    return fg


def _pack(fg, graphs):
    csrs = [oracle.canonical_csr(g.n, g.src, g.dst) for g in graphs]
    vtx, off, idx = fg.batch_pack(csrs)
    exp = np.concatenate([oracle.net(o, i) for o, i in csrs]) if csrs else np.zeros((0, 16), np.int64)
    return vtx, off, idx, exp


def _mixed():
    graphs = graphgen.batch_graphs(96, seed=21)
    graphs += [graphgen.clique(40), graphgen.star(300), graphgen.erdos_renyi(512, 0.3, seed=3),
               graphgen.cycle(16), graphgen.path(2), graphgen.clique(1), graphgen.clique(64),
               graphgen.clique(65)]
    return graphs


@pytest.mark.parametrize("threads", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("hub,bpc", [(0, 0), (-1, 0), (1, 1), (8, 2), (64, 64)])
def test_batch_mixed(fg, threads, hub, bpc):
    """Every plan: thread-per-vertex only (hub -1), every vertex by a
    wavefront (hub 1), mixed; the grid capped at 1, 2 or 64 workgroups per CU
    (never more workgroups than graphs)."""
    vtx, off, idx, exp = _pack(fg, _mixed())
    say(f"batch mixed threads={threads} hub={hub} bpc={bpc} G={int(vtx.numel()) - 1} n={int(vtx[-1])}")
    out = fg.batch(vtx, off.cuda(), idx.cuda(), plan={"threads": threads, "hub_degree": hub, "blocks_per_cu": bpc})
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), exp)


def test_batch_persistent_queue_and_tuner(fg):
    """512 graphs through 256 persistent workgroups (two rounds of the queue
    at least), and the autotuner: its plan gives the oracle's result, and a
    second call on a batch of the same shape and size histogram returns the
    cached plan."""
    graphs = graphgen.batch_graphs(512, seed=23)
    vtx, off, idx, exp = _pack(fg, graphs)
    o, i = off.cuda(), idx.cuda()
    say("batch 512 graphs, one workgroup per CU")
    out = fg.batch(vtx, o, i, plan={"blocks_per_cu": 1})
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), exp)
    say("batch tuner")
    plan = fg.batch_tune(vtx, o, i, reps=2)
    assert plan["threads"] in (128, 256, 512) and plan["blocks_per_cu"] in (2, 4, 8, 64)
    assert plan["hub_degree"] in (16, 32, 64, -1)
    np.testing.assert_array_equal(fg.batch(vtx, o, i, plan=plan).cpu().numpy(), exp)
    s = torch.cuda.Stream()  # graph capture needs a stream other than the legacy default one
    with torch.cuda.stream(s):
        got = fg.batch(vtx, o, i, plan=dict(plan, use_graph=1))
        s.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), exp)
    fg.batch_release(s)
    assert fg.batch_tune(vtx, o, i, reps=2) == plan


def test_batch_unsorted_rows(fg):
    """Rows in any order (the contract of fglt_raw, which the batch shares):
    the batch's rows shuffled per vertex give the oracle's counts."""
    vtx, off, idx, exp = _pack(fg, _mixed())
    rng = np.random.default_rng(12)
    o, ix = off.numpy(), idx.numpy().copy()
    for v in range(o.size - 1):
        a, b = int(o[v]), int(o[v + 1])
        if b - a > 1:
            ix[a:b] = ix[a:b][rng.permutation(b - a)]
    say("batch with shuffled rows")
    out = fg.batch(vtx, off.cuda(), torch.from_numpy(ix).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), exp)


def test_batch_matches_single_graph_path(fg):
    graphs = graphgen.batch_graphs(64, seed=22)
    vtx, off, idx, exp = _pack(fg, graphs)
    say("batch vs fglt_raw on the block-diagonal union")
    o, i = off.cuda(), idx.cuda()
    np.testing.assert_array_equal(fg.batch(vtx, o, i).cpu().numpy(), fg.transform(o, i).cpu().numpy())


def test_batch_graph_replay(fg):
    """The captured HIP graph is replayed with new arguments each call; eager
    work and synchronizations run between the replays."""
    s = torch.cuda.Stream()
    cases = []
    for seed in (31, 32, 33):
        graphs = graphgen.batch_graphs(50, seed=seed)
        cases.append(_pack(fg, graphs))
    with torch.cuda.stream(s):
        for rep in range(2):
            for k, (vtx, off, idx, exp) in enumerate(cases):
                say(f"graph replay rep={rep} case={k}")
                out = fg.batch(vtx, off.cuda(), idx.cuda(), plan={"use_graph": 1})
                torch.cuda.current_stream().synchronize()
                np.testing.assert_array_equal(out.cpu().numpy(), exp)
                _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
    fg._lib.lib().fglt_batch_release(ctypes.c_void_p(s.cuda_stream))


def test_batch_contract(fg):
    say("batch contract")
    big = graphgen.erdos_renyi(600, 0.01, seed=4)
    vtx, off, idx, _ = _pack(fg, [big])
    with pytest.raises(fg.FgltError) as e:
        fg.batch(vtx, off.cuda(), idx.cuda())
    assert e.value.status == -6
    # an asymmetric graph is skipped on the device and reported by fglt_batch_status
    off_a = torch.tensor([0, 1, 1], dtype=torch.int64)
    idx_a = torch.tensor([1], dtype=torch.int32)
    vtx_a = torch.tensor([0, 2], dtype=torch.int64)
    L = fg._lib.lib()
    ws = torch.empty(int(L.fglt_batch_workspace(1, 2, 1)), dtype=torch.uint8, device="cuda")
    fg.batch(vtx_a, off_a.cuda(), idx_a.cuda(), workspace=ws)
    st = L.fglt_batch_status(ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -2
    # a canonical batch leaves the status word clear
    vtx, off, idx, _ = _pack(fg, graphgen.batch_graphs(4, seed=5))
    ws2 = torch.empty(int(L.fglt_batch_workspace(4, int(vtx[-1]), int(idx.numel()))), dtype=torch.uint8, device="cuda")
    fg.batch(vtx, off.cuda(), idx.cuda(), workspace=ws2)
    assert L.fglt_batch_status(ctypes.c_void_p(ws2.data_ptr()),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0


def test_batch_rejects_offsets_outside_the_indices(fg):
    """Row offsets before 0 or past nnz_total are flagged on the device (the
    rows are skipped, the status word reads ENOTCANON) and never read."""
    L = fg._lib.lib()
    cases = [
        ("negative start", [0, 2], [-4, 1, 2], [1, 0]),
        ("end past the indices", [0, 2], [0, 1, 9], [1, 0]),
    ]
    for name, vtx, off, idx in cases:
        say(f"batch malformed offsets: {name}")
        vtx_t = torch.tensor(vtx, dtype=torch.int64)
        ws = torch.empty(int(L.fglt_batch_workspace(1, 2, len(idx))), dtype=torch.uint8, device="cuda")
        fg.batch(vtx_t, torch.tensor(off, dtype=torch.int64).cuda(), torch.tensor(idx, dtype=torch.int32).cuda(),
                 workspace=ws)
        assert fg.batch_status(ws) == -2, name


def test_server_fails_a_malformed_batched_request_alone(fg):
    from paper_2007_11111_amd.server import GpuExecutor, Server
    good = [oracle.canonical_csr(g.n, g.src, g.dst) for g in graphgen.batch_graphs(5, seed=41)]
    bad = (np.array([0, 1, 1], np.int64), np.array([1], np.int32))  # (0, 1) without (1, 0)
    reqs = good[:2] + [bad] + good[2:]
    say("server: a batch with one asymmetric request")
    srv = Server(GpuExecutor(), budget_bytes=1 << 30, streams=1)
    try:
        futs = [srv.submit(o, i) for o, i in reqs]
        for k, f in enumerate(futs):
            if k == 2:
                with pytest.raises(fg.FgltError):
                    f.result(timeout=60)
            else:
                r = f.result(timeout=60)
                np.testing.assert_array_equal(r.net.cpu().numpy(), oracle.net(*reqs[k]))
                r.release()
    finally:
        srv.close()
    assert srv.free == 1 << 30
