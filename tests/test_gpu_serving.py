"""Serving loop on the GPU: many integrals of different shapes advance
together, each with the result it has alone (within 1e-12), matching the
oracle in FP64 mode; admission by slots and by a device-memory budget."""
import numpy as np
import pytest

import tolerances as T
from paper_2010_09341_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2010_09341_amd import vegas
    vegas.lib()
    return vegas


def _submit(vg, srv, r: W.Request, prec=None):
    return vg.vegas_server_submit(srv, r.dim, r.nb, r.fid, r.params, r.n_events, r.n_iter,
                                  r.alpha, r.seed, r.prec if prec is None else prec)


def test_served_fp64_matches_oracle(vg, orc):
    srv = vg.vegas_server_create(1 << 28, 64)
    reqs = [W.Request(0, 0.0, 4, 50, W.F_GAUSS, [0.1], 100_000, 5, 1.5, 0, W.FP64),
            W.Request(1, 0.0, 3, 37, W.F_BW_FLAT, [0.42, 0.03], 20_011, 6, 1.5, 7, W.FP64),
            W.Request(2, 0.0, 20, 8, W.F_SUM, None, 9_999, 3, 1.5, 3, W.FP64),
            W.Request(3, 0.0, 4, 100, W.F_LO_TOY, [13000.0, 91.19, 2.5, 20.0], 50_000, 3,
                      1.5, 1, W.FP64)]
    tickets = [_submit(vg, srv, r) for r in reqs]
    for r, tk in zip(reqs, tickets):
        I, s, c2, lat = vg.vegas_server_wait(srv, tk, 120.0)
        I_t, s_t = vg.vegas_server_iterations(srv, tk, r.n_iter)
        I_r, s_r, _, _ = orc.run(r.dim, r.nb, r.fid, r.params, r.n_events, r.seed, r.n_iter,
                                 r.alpha)
        assert np.all(np.abs(I_t - I_r) <= 1e-12 * np.abs(I_r)), (r.index, I_t, I_r)
        assert T.sigma_close(s_t, s_r, I_r, r.n_events), T.sigma_excess(s_t, s_r, I_r, r.n_events)
        I_o, s_o, _ = orc.combine(I_r, s_r)
        assert T.combine_close(I, s, I_t, s_t, I_o, s_o, r.n_events), (I, I_o, s, s_o)
        assert lat > 0
    done, events, items, peak = vg.vegas_server_stats(srv)
    assert done == 4 and events == sum(r.n_events * r.n_iter for r in reqs)
    vg.vegas_server_destroy(srv)


def test_served_extreme_shapes_fp64(vg, orc):
    """The serving kernels at the shape limits, FP64 against the oracle: the
    cell maximum (32 dimensions x 256 bins, the 32-dimension class, one LDS
    histogram copy) and the minimum (1 dimension, 2 bins, 2 events), served
    together. At the cell maximum the Gaussian runs one iteration (on the
    uniform grid: the same events, weights and sums); the refinement at that
    shape is exercised by three iterations of the sum integrand, whose
    per-dimension w^2 histograms are smooth. (A 32-dimension Gaussian refined
    from 2e4 events leaves bins whose compressed weights r_k are tiny; the
    refined edges then carry the amplified rounding-order difference that the
    edge bound of the parity tests describes, and its third iteration read
    2e-12 from the oracle's.)"""
    srv = vg.vegas_server_create(1 << 28, 8)
    reqs = [W.Request(0, 0.0, 32, 256, W.F_GAUSS, [0.3], 20_011, 1, 1.5, 5, W.FP64),
            W.Request(1, 0.0, 32, 256, W.F_SUM, None, 100_003, 3, 1.5, 8, W.FP64),
            W.Request(2, 0.0, 1, 2, W.F_GAUSS, [0.3], 2, 4, 1.5, 6, W.FP64),
            W.Request(3, 0.0, 17, 31, W.F_SUM, None, 7_777, 2, 0.5, 7, W.FP64)]
    tickets = [_submit(vg, srv, r) for r in reqs]
    for r, tk in zip(reqs, tickets):
        vg.vegas_server_wait(srv, tk, 120.0)
        I_t, s_t = vg.vegas_server_iterations(srv, tk, r.n_iter)
        I_r, s_r, _, _ = orc.run(r.dim, r.nb, r.fid, r.params, r.n_events, r.seed, r.n_iter,
                                 r.alpha)
        assert np.all(np.abs(I_t - I_r) <= 1e-12 * np.abs(I_r)), (r.index, I_t, I_r)
        assert T.sigma_close(s_t, s_r, I_r, r.n_events), (r.index,
                                                           T.sigma_excess(s_t, s_r, I_r, r.n_events))
        vg.vegas_server_release(srv, tk)
    vg.vegas_server_destroy(srv)


def test_alone_equals_in_the_mix(vg):
    """20 requests from the serving trace, each run alone on its own server,
    then all 200 trace requests together: the 20 agree within 1e-12."""
    trace = W.serving_trace(200, rate_per_s=1e9, seed=3, max_events=300_000)
    picks = trace[::10]
    alone = {}
    for r in picks:
        srv = vg.vegas_server_create(1 << 28, 4)
        tk = _submit(vg, srv, r)
        vg.vegas_server_wait(srv, tk, 120.0)
        alone[r.index] = vg.vegas_server_iterations(srv, tk, r.n_iter)
        vg.vegas_server_destroy(srv)
    srv = vg.vegas_server_create(1 << 30, 256)
    tickets = {r.index: _submit(vg, srv, r) for r in trace}
    for r in trace:
        vg.vegas_server_wait(srv, tickets[r.index], 300.0)
    for r in picks:
        I_t, s_t = vg.vegas_server_iterations(srv, tickets[r.index], r.n_iter)
        I_a, s_a = alone[r.index]
        assert np.all(np.abs(I_t - I_a) <= 1e-12 * np.abs(I_a)), (r.index, I_t - I_a)
        assert T.sigma_close(s_t, s_a, I_a, r.n_events), T.sigma_excess(s_t, s_a, I_a, r.n_events)
    done, events, items, peak = vg.vegas_server_stats(srv)
    assert done == len(trace)
    assert peak > 1  # requests overlapped on the device
    vg.vegas_server_destroy(srv)


def test_served_closed_forms(vg):
    trace = W.serving_trace(40, rate_per_s=1e9, seed=5, max_events=1_000_000)
    srv = vg.vegas_server_create(1 << 28, 16)
    tickets = [_submit(vg, srv, r) for r in trace]
    pulls = []
    for r, tk in zip(trace, tickets):
        I, s, c2, _ = vg.vegas_server_wait(srv, tk, 120.0)
        # first iterations on the uniform grid are the least precise; the
        # combined estimate must still sit on the closed form
        pulls.append((I - W.request_closed_form(r)) / s)
    pulls = np.array(pulls)
    assert np.mean(np.abs(pulls) < 4) > 0.9
    vg.vegas_server_destroy(srv)


def test_admission_by_memory_and_slots(vg):
    """A budget that holds at most two of these integrals at a time, and a
    request larger than the whole budget."""
    from paper_2010_09341_amd.vegas import vegas_workspace_bytes
    # a handle's workspace (4096 partial slots, 1024 result entries) is a bit
    # more than twice a served 12 x 100 integral with 5 chunks and 4 iterations
    budget = vegas_workspace_bytes(12, 100)
    srv = vg.vegas_server_create(budget, 64)
    reqs = [W.Request(i, 0.0, 12, 100, W.F_GAUSS, [0.2], 20_000, 4, 1.5, i, W.FP32_EVAL)
            for i in range(8)]
    tks = [_submit(vg, srv, r) for r in reqs]
    for tk in tks:
        vg.vegas_server_wait(srv, tk, 120.0)
    done, _, _, peak = vg.vegas_server_stats(srv)
    assert done == 8 and 1 <= peak <= 2
    vg.vegas_server_destroy(srv)
    # with a fixed chunk of 2048 events, the partial slots of 1e10 events per
    # iteration alone exceed the budget
    srv = vg.vegas_server_create(budget, 64, 2048)
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_server_submit(srv, 12, 100, W.F_GAUSS, [0.2], 10**10, 4, 1.5, 0)
    assert e.value.code == vg.VEGAS_ENOMEM
    vg.vegas_server_destroy(srv)
    srv = vg.vegas_server_create(1 << 28, 2)
    tks = [_submit(vg, srv, r) for r in reqs]
    for tk in tks:
        vg.vegas_server_wait(srv, tk, 120.0)
    assert vg.vegas_server_stats(srv)[3] == 2
    vg.vegas_server_destroy(srv)


def test_release(vg):
    """A finished ticket's record is freed by vegas_server_release; reading
    it afterwards, releasing it twice or an unknown ticket is VEGAS_EINVAL; a
    ticket still queued (one slot, held by a request of 10 x 5e7 events, a
    few milliseconds of device work, while the release follows the submission
    within microseconds) is VEGAS_EBUSY; the other tickets are untouched."""
    srv = vg.vegas_server_create(1 << 28, 1)
    long_r = W.Request(0, 0.0, 8, 50, W.F_GAUSS, [0.1], 50_000_000, 10, 1.5, 1, W.FP32_EVAL)
    short = W.Request(1, 0.0, 3, 20, W.F_GAUSS, [0.2], 10_000, 3, 1.5, 2, W.FP64)
    tk_long = _submit(vg, srv, long_r)
    tk_a = _submit(vg, srv, short)
    tk_b = _submit(vg, srv, short)
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_server_release(srv, tk_b)
    assert e.value.code == vg.VEGAS_EBUSY
    for tk in (tk_long, tk_a, tk_b):
        vg.vegas_server_wait(srv, tk, 120.0)
    I_b, s_b, _, _ = vg.vegas_server_wait(srv, tk_b, 0.0)
    vg.vegas_server_release(srv, tk_a)
    for call in (lambda: vg.vegas_server_wait(srv, tk_a, 0.0),
                 lambda: vg.vegas_server_iterations(srv, tk_a, short.n_iter),
                 lambda: vg.vegas_server_release(srv, tk_a),
                 lambda: vg.vegas_server_release(srv, 10**9)):
        with pytest.raises(vg.VegasError) as e:
            call()
        assert e.value.code == vg.VEGAS_EINVAL
    # the same request in another ticket is unaffected
    assert vg.vegas_server_wait(srv, tk_b, 0.0)[:2] == (I_b, s_b)
    vg.vegas_server_release(srv, tk_b)
    vg.vegas_server_release(srv, tk_long)
    vg.vegas_server_destroy(srv)


def test_release_while_another_thread_waits(vg):
    """A ticket released by one thread while another thread waits on it: the
    waiter returns the result (it read it first) or VEGAS_EINVAL (the release
    came first), never a freed record; 24 rounds at different timings."""
    import threading
    srv = vg.vegas_server_create(1 << 28, 4)
    outcomes = []
    for i in range(24):
        r = W.Request(i, 0.0, 4, 30, W.F_GAUSS, [0.2], 20_000 + 5_000 * (i % 6), 3, 1.5, i,
                      W.FP32_EVAL)
        tk = _submit(vg, srv, r)
        got = []

        def waiter(tk=tk, got=got):
            try:
                got.append(("ok", vg.vegas_server_wait(srv, tk, 60.0)[:2]))
            except vg.VegasError as e:
                got.append(("err", e.code))

        t = threading.Thread(target=waiter)
        t.start()
        ref = vg.vegas_server_wait(srv, tk, 60.0)[:2]
        vg.vegas_server_release(srv, tk)
        t.join(timeout=60.0)
        assert not t.is_alive() and len(got) == 1
        kind, val = got[0]
        assert (kind == "ok" and val == ref) or (kind == "err" and val == vg.VEGAS_EINVAL), got
        outcomes.append(kind)
    vg.vegas_server_destroy(srv)
    assert len(outcomes) == 24


def test_concurrent_clients(vg):
    """Server calls from several threads at once (the library's calls
    release the interpreter lock): four threads each submit, wait for and
    release 12 trace requests, interleaved with each other and with a
    statistics reader; every result agrees with the same request served alone
    as in the mix test (same chunks and partial slots; the refined grids
    agree to rounding, the histogram being summed with atomics)."""
    import threading
    trace = W.serving_trace(48, rate_per_s=1e9, seed=11, max_events=200_000)
    alone = {}
    for r in trace[::6]:
        srv = vg.vegas_server_create(1 << 28, 4)
        tk = _submit(vg, srv, r)
        alone[r.index] = vg.vegas_server_wait(srv, tk, 120.0)[:2]
        vg.vegas_server_destroy(srv)
    srv = vg.vegas_server_create(1 << 28, 16)
    got, errors = {}, []

    def client(part):
        try:
            mine = [(r, _submit(vg, srv, r)) for r in part]
            for r, tk in mine:
                got[r.index] = vg.vegas_server_wait(srv, tk, 120.0)[:2]
                vg.vegas_server_release(srv, tk)
                vg.vegas_server_stats(srv)
        except Exception as e:  # noqa: BLE001 - reported by the assertion below
            errors.append(repr(e))

    threads = [threading.Thread(target=client, args=(trace[i::4],)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=180.0)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    assert sorted(got) == [r.index for r in trace]
    by_index = {r.index: r for r in trace}
    for i, (I_a, s_a) in alone.items():
        I_g, s_g = got[i]
        assert abs(I_g - I_a) <= 1e-12 * abs(I_a), (i, I_g, I_a)
        assert T.sigma_close(s_g, s_a, I_a, by_index[i].n_events), (i, s_g, s_a)
    assert vg.vegas_server_stats(srv)[0] == len(trace)
    vg.vegas_server_destroy(srv)


def test_served_matches_handle(vg):
    """The serving path and the single-integral path compute the same
    iterations (different launch shapes: agreement to rounding)."""
    r = W.Request(0, 0.0, 8, 50, W.F_GAUSS, [0.1], 1_000_000, 4, 1.5, 11, W.FP32_EVAL)
    srv = vg.vegas_server_create(1 << 28, 8)
    tk = _submit(vg, srv, r)
    vg.vegas_server_wait(srv, tk, 120.0)
    I_s, s_s = vg.vegas_server_iterations(srv, tk, r.n_iter)
    vg.vegas_server_destroy(srv)
    h = vg.vegas_create(8, 50)
    vg.vegas_set_params(h, W.F_GAUSS, [0.1])
    vg.vegas_set_precision(h, W.FP32_EVAL)
    I_h, s_h = vg.vegas_run(h, W.F_GAUSS, r.n_events, r.seed, r.n_iter, r.alpha)
    assert np.all(np.abs(I_s - I_h) <= 1e-12 * np.abs(I_h))


def test_submit_validation(vg):
    srv = vg.vegas_server_create(1 << 24, 4)
    bad = [dict(dim=0), dict(n_bins=1), dict(n_events=1), dict(n_iter=0), dict(alpha=-1.0),
           dict(integrand_id=99), dict(prec=7), dict(integrand_id=W.F_LO_TOY)]
    base = dict(dim=3, n_bins=10, integrand_id=W.F_GAUSS, params=[0.2], n_events=1000,
                n_iter=2, alpha=1.5, seed=0, prec=W.FP64)
    for b in bad:
        kw = dict(base)
        kw.update(b)
        with pytest.raises(vg.VegasError) as e:
            vg.vegas_server_submit(srv, **kw)
        assert e.value.code == vg.VEGAS_EINVAL, b
    vg.vegas_server_destroy(srv)


def test_graph_replayed_ticks(vg, orc):
    """Ticks that repeat the previous tick's work are replayed from a captured
    hipGraph when enabled: with replays on and off, three FP64 integrals of 20
    iterations match the oracle at 1e-12, and replays happen only when on."""
    reqs = [W.Request(0, 0.0, 5, 40, W.F_GAUSS, [0.15], 60_000, 20, 1.5, 2, W.FP64),
            W.Request(1, 0.0, 2, 64, W.F_BW_FLAT, [0.3, 0.05], 30_001, 20, 1.5, 9, W.FP64),
            W.Request(2, 0.0, 18, 10, W.F_GAUSS, [0.3], 8_191, 20, 1.5, 4, W.FP64)]
    ref = [orc.run(r.dim, r.nb, r.fid, r.params, r.n_events, r.seed, r.n_iter, r.alpha)
           for r in reqs]
    for graph in (True, False):
        srv = vg.vegas_server_create(1 << 28, 8)
        vg.vegas_server_set_graph(srv, graph)
        tickets = [_submit(vg, srv, r) for r in reqs]
        for r, tk, (I_r, s_r, _, _) in zip(reqs, tickets, ref):
            vg.vegas_server_wait(srv, tk, 120.0)
            I_t, s_t = vg.vegas_server_iterations(srv, tk, r.n_iter)
            assert np.all(np.abs(I_t - I_r) <= 1e-12 * np.abs(I_r)), (graph, r.index, I_t - I_r)
            assert T.sigma_close(s_t, s_r, I_r, r.n_events), \
                T.sigma_excess(s_t, s_r, I_r, r.n_events)
        ticks, graph_ticks = vg.vegas_server_ticks(srv)
        assert ticks >= 20
        if graph:
            assert graph_ticks >= 5, (ticks, graph_ticks)
        else:
            assert graph_ticks == 0
        vg.vegas_server_destroy(srv)


def test_large_requests_use_the_iteration_kernel(vg, orc):
    """Requests of at least 2^20 events per iteration run as launches of the
    single-integral iteration kernel: FP64 matches the oracle at 1e-12, and
    the result is the same alone, in a mix of small and large requests, and
    through the handle path."""
    big64 = W.Request(0, 0.0, 6, 40, W.F_GAUSS, [0.2], 2_000_003, 4, 1.5, 21, W.FP64)
    big32 = W.Request(1, 0.0, 4, 100, W.F_LO_TOY, [13000.0, 91.19, 2.5, 20.0], 1_500_000, 3,
                      1.5, 5, W.FP32_EVAL)
    small = W.serving_trace(30, rate_per_s=1e9, seed=11, max_events=200_000)
    I_r, s_r, _, _ = orc.run(big64.dim, big64.nb, big64.fid, big64.params, big64.n_events,
                             big64.seed, big64.n_iter, big64.alpha)
    res = {}
    for mix in (False, True):
        srv = vg.vegas_server_create(1 << 30, 64)
        reqs = ([big64, big32] + list(small)) if mix else [big64, big32]
        tickets = [_submit(vg, srv, r) for r in reqs]
        for tk in tickets:
            vg.vegas_server_wait(srv, tk, 300.0)
        res[mix] = [vg.vegas_server_iterations(srv, tickets[i], reqs[i].n_iter) for i in (0, 1)]
        vg.vegas_server_destroy(srv)
    I_a, s_a = res[False][0]
    assert np.all(np.abs(I_a - I_r) <= 1e-12 * np.abs(I_r)), (I_a - I_r) / I_r
    assert T.sigma_close(s_a, s_r, I_r, big64.n_events), T.sigma_excess(s_a, s_r, I_r, big64.n_events)
    for i in (0, 1):
        (Ia, sa), (Im, sm) = res[False][i], res[True][i]
        assert np.all(np.abs(Im - Ia) <= 1e-13 * np.abs(Ia)), (i, Im - Ia)
        assert T.sigma_close(sm, sa, Ia, reqs[i].n_events)
    h = vg.vegas_create(big32.dim, big32.nb)
    vg.vegas_set_params(h, big32.fid, big32.params)
    vg.vegas_set_precision(h, big32.prec)
    I_h, s_h = vg.vegas_run(h, big32.fid, big32.n_events, big32.seed, big32.n_iter, big32.alpha)
    assert np.all(np.abs(res[False][1][0] - I_h) <= 1e-13 * np.abs(I_h))


def test_chained_ticks(vg, orc):
    """The ticks up to the next completion run as one chain with one host
    synchronisation: three FP64 integrals of 7, 12 and 20 iterations need
    three chains (one per completion), match the oracle at the FP64 bounds,
    and agree with the same server synchronising after every tick; a request
    submitted while a chain runs is admitted after it and matches too."""
    reqs = [W.Request(0, 0.0, 5, 40, W.F_GAUSS, [0.15], 60_000, 7, 1.5, 2, W.FP64),
            W.Request(1, 0.0, 2, 64, W.F_BW_FLAT, [0.3, 0.05], 30_001, 12, 1.5, 9, W.FP64),
            W.Request(2, 0.0, 18, 10, W.F_GAUSS, [0.3], 8_191, 20, 1.5, 4, W.FP64)]
    late = W.Request(3, 0.0, 3, 25, W.F_GAUSS, [0.2], 40_000, 6, 1.5, 8, W.FP64)
    ref = [orc.run(r.dim, r.nb, r.fid, r.params, r.n_events, r.seed, r.n_iter, r.alpha)
           for r in reqs + [late]]
    got = {}
    for chain in (32, 1):
        srv = vg.vegas_server_create(1 << 28, 8)
        vg.vegas_server_set_chain(srv, chain)
        tickets = [_submit(vg, srv, r) for r in reqs]
        vg.vegas_server_wait(srv, tickets[0], 120.0)
        tickets.append(_submit(vg, srv, late))
        for r, tk, (I_r, s_r, _, _) in zip(reqs + [late], tickets, ref):
            vg.vegas_server_wait(srv, tk, 120.0)
            I_t, s_t = vg.vegas_server_iterations(srv, tk, r.n_iter)
            assert np.all(np.abs(I_t - I_r) <= 1e-12 * np.abs(I_r)), (chain, r.index, I_t - I_r)
            assert T.sigma_close(s_t, s_r, I_r, r.n_events), \
                T.sigma_excess(s_t, s_r, I_r, r.n_events)
            got[chain, r.index] = I_t
        ticks, _ = vg.vegas_server_ticks(srv)
        chains = vg.vegas_server_chains(srv)
        if chain == 1:
            assert chains == ticks
        else:
            # 7 + 5 + 8 ticks for the first three, then the late request's
            # ticks, in at most a handful of chains
            assert chains <= 8 and ticks >= 20, (chains, ticks)
        vg.vegas_server_destroy(srv)
    for r in reqs + [late]:
        assert np.all(np.abs(got[32, r.index] - got[1, r.index]) <= 1e-12 *
                      np.abs(got[1, r.index]))
    srv = vg.vegas_server_create(1 << 24, 4)
    for bad in (0, 33):
        with pytest.raises(vg.VegasError) as e:
            vg.vegas_server_set_chain(srv, bad)
        assert e.value.code == vg.VEGAS_EINVAL
    vg.vegas_server_destroy(srv)


def test_lanes(vg, orc):
    """Chains run on up to 8 streams (lanes): with one lane and with four,
    six FP64 integrals submitted together match the oracle at the FP64
    bounds, and with four lanes they run in at least two lanes' chains at
    once; the lane count is rejected outside 1..8 and while requests are in
    flight."""
    reqs = [W.Request(i, 0.0, 2 + i, 20 + 7 * i, W.F_GAUSS, [0.2], 30_000 + 1_000 * i, 4 + i,
                      1.5, 100 + i, W.FP64) for i in range(6)]
    ref = [orc.run(r.dim, r.nb, r.fid, r.params, r.n_events, r.seed, r.n_iter, r.alpha)
           for r in reqs]
    for lanes in (1, 4):
        srv = vg.vegas_server_create(1 << 28, 16)
        vg.vegas_server_set_lanes(srv, lanes)
        tickets = [_submit(vg, srv, r) for r in reqs]
        for r, tk, (I_r, s_r, _, _) in zip(reqs, tickets, ref):
            vg.vegas_server_wait(srv, tk, 120.0)
            I_t, s_t = vg.vegas_server_iterations(srv, tk, r.n_iter)
            assert np.all(np.abs(I_t - I_r) <= 1e-12 * np.abs(I_r)), (lanes, r.index, I_t - I_r)
            assert T.sigma_close(s_t, s_r, I_r, r.n_events), \
                T.sigma_excess(s_t, s_r, I_r, r.n_events)
        vg.vegas_server_destroy(srv)
    srv = vg.vegas_server_create(1 << 28, 16)
    for bad in (0, 9):
        with pytest.raises(vg.VegasError) as e:
            vg.vegas_server_set_lanes(srv, bad)
        assert e.value.code == vg.VEGAS_EINVAL
    big = W.Request(0, 0.0, 8, 50, W.F_GAUSS, [0.1], 3_000_000, 10, 1.5, 1, W.FP32_EVAL)
    tk = _submit(vg, srv, big)
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_server_set_lanes(srv, 2)
    assert e.value.code == vg.VEGAS_ESTATE
    vg.vegas_server_wait(srv, tk, 120.0)
    vg.vegas_server_set_lanes(srv, 2)
    vg.vegas_server_destroy(srv)
