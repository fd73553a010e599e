"""GPU serving loop: resident data sets, continuous batching of requests of
mixed sizes over several streams; every result is bitwise identical to the
same request run alone, and matches the FP64 oracle."""
import numpy as np
import pytest

import synth
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import torch
    assert torch.cuda.is_available()
    import paper_2407_07096_amd as s
    s.load()
    return s


def test_alone_vs_mixed_bitwise(stag, orc):
    import torch
    rng = np.random.default_rng(0)
    datasets = []
    for k, (n, d, form) in enumerate([(20_000, 16, "fp32"), (30_000, 64, "fp16_split"), (9_000, 256, "bf16_split3")]):
        mix = synth.mixture(d, 10, 4000 + k, sigma=(0.5, 2.0))
        X = synth.sample(mix, n, 5000 + k)
        datasets.append((X, mix, 0.64 / d, form))
    # one stream: requests queue behind the running batch and get packed
    srv = stag.Server(budget_bytes=1 << 30, n_streams=1, max_batch_queries=20000)
    ids = [srv.add_dataset(to_dev(X), a, form) for X, _, a, form in datasets]
    srv4 = stag.Server(budget_bytes=1 << 30, n_streams=4, max_batch_queries=20000)
    ids4 = [srv4.add_dataset(to_dev(X), a, form) for X, _, a, form in datasets]
    sizes = [1, 3, 130, 2000, 17, 5000, 64, 1, 999, 4096, 7, 300]
    reqs = []
    for r, m in enumerate(sizes):
        k = r % 3
        X, mix, a, form = datasets[k]
        Q = synth.sample(mix, m, 6000 + r)
        reqs.append((k, Q))
    announce("serve mixed: 12 requests over 3 data sets")
    tickets = [srv.submit(ids[k], to_dev(Q)) for k, Q in reqs]
    mixed = []
    for t in tickets:
        S, st, lat = srv.wait(t)
        assert st == 0
        mixed.append(S.clone())
    st = srv.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0
    assert st["batches"] < len(sizes)  # requests were packed together
    # the same requests alone, one at a time, on the four-stream server
    for (k, Q), Sm in zip(reqs, mixed):
        t = srv4.submit(ids4[k], to_dev(Q))
        Sa, st, _ = srv4.wait(t)
        assert st == 0
        assert torch.equal(Sa, Sm)
    # and all at once on the four-stream server (concurrent batches)
    tickets = [srv4.submit(ids4[k], to_dev(Q)) for k, Q in reqs]
    for t, Sm in zip(tickets, mixed):
        Sc, st, _ = srv4.wait(t)
        assert st == 0 and torch.equal(Sc, Sm)
    # and equal to the one-shot API
    for (k, Q), Sm in zip(reqs, mixed):
        X, _, a, form = datasets[k]
        S1 = stag.kde_exact(to_dev(X), to_dev(Q), a, form=form)
        torch.cuda.synchronize()
        assert torch.equal(S1, Sm)
    # accuracy against the oracle on a few requests
    for (k, Q), Sm in list(zip(reqs, mixed))[:6]:
        X, _, a, form = datasets[k]
        ref = orc.kde_exact(X, Q, a)
        err = np.abs(Sm.cpu().numpy() - ref) / ref
        assert err.max() < 1e-4
    srv.close()
    srv4.close()


def test_rejects_oversized_request(stag):
    import torch
    X, Q, _ = synth.config_points(2, n=5000, m=2000)
    srv = stag.Server(budget_bytes=1 << 18, n_streams=2)
    i = srv.add_dataset(to_dev(X), 0.01)
    t = srv.submit(i, to_dev(Q))
    S, st, _ = srv.wait(t)
    assert st == 5  # STAG_E_BUSY
    t = srv.submit(i, to_dev(Q[:10].copy()))
    S, st, _ = srv.wait(t)
    assert st == 0
    srv.close()


def test_forms_auto_lsh_and_chunks(stag, orc):
    """Data sets resident in fp32 (centred) and bf16 split with a CKNS index:
    exact requests in explicit forms and in STAG_FORM_AUTO (the form chosen
    from eps among the resident ones), and LSH requests answered by the
    resident index, chunked (512 queries) and mixed over four streams.  Every
    result is bitwise equal to the same request alone on a one-stream server
    without chunking, to the one-shot call (stag_kde_exact in the chosen
    form; the index's own query for LSH), and within its bound of the
    oracle."""
    import torch
    dsets = []
    for k, (n, d) in enumerate([(12_000, 16), (20_000, 64)]):
        mix = synth.mixture(d, 10, 4100 + k, sigma=(0.5, 2.0))
        X = synth.sample(mix, n, 5100 + k)
        dsets.append((X, mix, 0.64 / d))
    lsh = dict(eps=0.5, k1=2, k2_constant=6, p_offset=1, seed=77)
    srv = stag.Server(budget_bytes=4 << 30, n_streams=4, max_batch_queries=8192, chunk_queries=512)
    one = stag.Server(budget_bytes=4 << 30, n_streams=1, max_batch_queries=1 << 20, chunk_queries=1 << 20)
    ids = [srv.add_dataset(to_dev(X), a, ["fp32", "bf16_split"], lsh=lsh) for X, _, a in dsets]
    ids1 = [one.add_dataset(to_dev(X), a, ["fp32", "bf16_split"], lsh=lsh) for X, _, a in dsets]
    # (data set, size, kind): explicit fp32 / bf16 split, AUTO at a loose and a
    # tight eps (bf16 split, then fp32), LSH
    plan = [(0, 3000, ("fp32", 0.0)), (1, 7, ("auto", 1e-2)), (0, 1500, "lsh"), (1, 2600, ("bf16_split", 0.0)),
            (0, 1, ("auto", 1e-12)), (1, 513, "lsh"), (0, 64, ("auto", 1e-2)), (1, 4000, ("auto", 1e-12)),
            (1, 1, "lsh"), (0, 900, ("bf16_split", 0.0))]
    reqs = []
    for r, (k, m, kind) in enumerate(plan):
        reqs.append((k, to_dev(synth.sample(dsets[k][1], m, 6100 + r)), kind))

    def submit(server, idl, k, Q, kind):
        if kind == "lsh":
            return server.submit(idl[k], Q, lsh=True)
        form, eps = kind
        return server.submit(idl[k], Q, form=form, eps=eps, bound=True)

    announce("serve forms/auto/lsh mixed over 4 streams, chunks of 512")
    tickets = [submit(srv, ids, k, Q, kind) for k, Q, kind in reqs]
    forms = [srv.form_of(t) for t in tickets]
    assert forms[1] == "bf16_split" and forms[4] == "fp32" and forms[7] == "fp32" and forms[2] is None
    mixed = []
    for t in tickets:
        S, st, _ = srv.wait(t)
        assert st == 0
        mixed.append((S.clone(), srv.bound_of(t)))
    assert srv.stats()["batches"] > len(plan)  # the large requests went in chunks
    for (k, Q, kind), (Sm, Bm), form in zip(reqs, mixed, forms):
        t = submit(one, ids1, k, Q, kind)
        Sa, st, _ = one.wait(t)
        assert st == 0 and torch.equal(Sa, Sm)
        X, _, a = dsets[k]
        if kind == "lsh":
            idx = stag.LshIndex(to_dev(X), a, **lsh)
            S1 = idx.query(Q)
            idx.close()
            torch.cuda.synchronize()
            assert torch.equal(S1, Sm)
        else:
            S1, B1 = stag.kde_exact(to_dev(X), Q, a, form=form, return_bound=True)
            torch.cuda.synchronize()
            assert torch.equal(S1, Sm)
            ref = orc.kde_exact(X, Q.cpu().numpy(), a)
            err = np.abs(Sm.cpu().numpy() - ref) / ref
            assert np.all(err <= Bm.cpu().numpy())
    srv.close()
    one.close()
