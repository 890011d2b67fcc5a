"""Serving by continuous batching (sfls_server_*): results are the same for a
request alone and in a mix whose members arrive while others are on the
device, admission follows pool memory and slots, the request loop runs
several size-class servers concurrently, and served estimates agree with the
oracle estimator."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_06073_amd as sf  # noqa: E402
from oracle.estimator import Params, estimate  # noqa: E402
from paper_1705_06073_amd import serving, synth  # noqa: E402
from tests import metrics  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx():
    c = sf.Context(0)
    yield c
    c.close()


def signals(ns, seed=0):
    """Requests of the serving recipe (K ~ Poisson(N/64), separation 1/N,
    alpha ~ CN(0,1), SNR ~ U[5,30] dB, complex64) at the given lengths."""
    out = []
    for i, N in enumerate(ns):
        rng = np.random.Generator(np.random.PCG64(synth.seed_for(9, 100 * seed + i)))
        K = int(rng.poisson(N / 64.0))
        snr = float(rng.uniform(5.0, 30.0))
        out.append(synth.make_instance(rng, int(N), K, 1.0 / N, "cn", snr, np.complex64))
    return out


def to_device(insts):
    """All signals in one device buffer; returns (tensor, byte addresses)."""
    y = np.concatenate([i.y.astype(np.complex64) for i in insts])
    t = torch.from_numpy(y.view(np.float32).copy()).to(DEV)
    base, addr, o = t.data_ptr(), [], 0
    for i in insts:
        addr.append(base + 8 * o)
        o += i.N
    return t, addr


def run_alone(srv, insts, addr):
    res = []
    for k, inst in enumerate(insts):
        assert srv.submit(addr[k], inst.N, k)
        got = []
        for _ in range(100000):
            srv.step()
            got += srv.poll()
            if got:
                break
        assert len(got) == 1 and got[0].tag == k
        res.append(got[0])
    return res


def run_mix(srv, insts, addr, waves):
    """Submit in waves between rounds (a request that finds no slot or memory
    waits for the next round); returns results by tag."""
    pending = []
    out = {}
    order = list(range(len(insts)))
    rounds = 0
    while len(out) < len(insts):
        if order and (rounds in waves or not pending and srv.stats()["in_flight"] == 0):
            take = order[:max(1, len(order) // 3)]
            pending += take
            order = order[len(take):]
        while pending and srv.submit(addr[pending[0]], insts[pending[0]].N, pending[0]):
            pending.pop(0)
        srv.step()
        rounds += 1
        for r in srv.poll():
            out[r.tag] = r
        assert rounds < 100000
    return [out[k] for k in range(len(insts))]


def same(a, b):
    assert a.K == b.K, (a.tag, a.K, b.K)
    assert a.status == b.status and a.iterations == b.iterations and a.evaluations == b.evaluations
    np.testing.assert_array_equal(a.theta, b.theta)
    np.testing.assert_array_equal(a.gamma, b.gamma)
    np.testing.assert_array_equal(a.alpha, b.alpha)
    assert a.beta == b.beta and a.zeta == b.zeta and a.objective == b.objective


@pytest.mark.parametrize("prec", [sf.SFLS_MIXED, sf.SFLS_FP64])
def test_results_same_alone_and_in_the_mix(ctx, prec):
    """Every request's estimate is bit-identical alone and in a mix of lengths
    whose members are admitted while earlier ones are mid-solve."""
    ns = [256, 1024, 300, 64, 700, 1024, 128, 512, 256, 1000, 96, 2048]
    insts = signals(ns)
    y, addr = to_device(insts)
    p = sf.default_params(precision=prec)
    srv = sf.Server(ctx, max_n=2048, max_slots=6, hbm_bytes=1 << 30, params=p)
    try:
        alone = run_alone(srv, insts, addr)
        mixed = run_mix(srv, insts, addr, waves={0, 3, 7, 12})
        st = srv.stats()
    finally:
        srv.close()
    for k, (a, b) in enumerate(zip(alone, mixed)):
        print(f"request {k}: N={insts[k].N} K={a.K} evals={a.evaluations}", flush=True)
        assert a.status in (sf.SFLS_OK, sf.SFLS_NOTCONV)
        same(a, b)
    assert st["completed"] == 2 * len(insts) and st["in_flight"] == 0 and st["units_used"] == 0


def test_served_estimates_match_the_oracle(ctx):
    """FP64 path: the served estimate of small requests has the oracle's model
    order and frequencies within 1e-9/N (signals with 3-5 components at 20 dB:
    a pure-noise request overfits to a flat objective, where the frequencies
    of the spurious components are not determined to that level)."""
    insts = [synth.workload_n64(7)]
    for i, (N, K) in enumerate([(128, 4), (200, 5)]):
        rng = np.random.Generator(np.random.PCG64(synth.seed_for(9, 900 + i)))
        insts.append(synth.make_instance(rng, N, K, 2.0 / N, "cn", 20.0, np.complex64))
    for inst in insts:
        inst.y = inst.y.astype(np.complex64)
    y, addr = to_device(insts)
    p = sf.default_params(precision=sf.SFLS_FP64)
    srv = sf.Server(ctx, max_n=256, max_slots=4, hbm_bytes=256 << 20, params=p)
    try:
        got = run_mix(srv, insts, addr, waves={0})
    finally:
        srv.close()
    for inst, g in zip(insts, got):
        o = estimate(inst.y.astype(np.complex128), Params())
        print(f"N={inst.N}: served K={g.K} oracle K={o.K}", flush=True)
        assert g.K == o.K
        if g.K:
            d = metrics.wrap_distance(g.theta, o.theta)
            assert np.max(d) < 1e-9 / inst.N, np.max(d) * inst.N
        assert abs(g.beta - o.beta) <= 1e-8 * o.beta


def test_admission_by_pool_memory_and_slots(ctx):
    """A pool that holds two N=1024 blocks admits two such requests, refuses a
    third (and anything else) until a round frees a block; a full slot table
    refuses as well."""
    probe = sf.Server(ctx, max_n=1024, max_slots=8, hbm_bytes=256 << 20)
    st = probe.stats()
    bpu, fixed = st["bytes_per_unit"], st["bytes_reserved"] - st["units_total"] * st["bytes_per_unit"]
    assert probe.footprint(1024) == 1024 * bpu and probe.footprint(700) == 1024 * bpu
    assert probe.footprint(10) == 64 * bpu
    probe.close()
    insts = signals([1024, 1024, 1024, 256], seed=2)
    y, addr = to_device(insts)
    srv = sf.Server(ctx, max_n=1024, max_slots=8, hbm_bytes=fixed + 3000 * bpu)
    try:
        assert srv.stats()["units_total"] == 2048
        assert srv.submit(addr[0], 1024, 0) and srv.submit(addr[1], 1024, 1)
        assert not srv.submit(addr[2], 1024, 2)
        assert not srv.submit(addr[3], 256, 3)
        assert srv.stats()["units_used"] == 2048
        done = []
        while not done:
            srv.step()
            done = srv.poll()
        assert srv.submit(addr[3], 256, 3)  # a freed block takes the small request
        while srv.stats()["in_flight"]:
            srv.step()
        srv.poll()
    finally:
        srv.close()
    srv = sf.Server(ctx, max_n=1024, max_slots=2, hbm_bytes=256 << 20)
    try:
        assert srv.submit(addr[3], 256, 0) and srv.submit(addr[3], 256, 1)
        assert not srv.submit(addr[3], 256, 2)
    finally:
        srv.close()


def test_bad_requests_are_rejected(ctx):
    insts = signals([512], seed=3)
    y, addr = to_device(insts)
    srv = sf.Server(ctx, max_n=256, max_slots=2, hbm_bytes=64 << 20)
    try:
        with pytest.raises(sf.SflsError) as e:
            srv.submit(addr[0], 512, 0)
        assert e.value.status == sf.SFLS_EUNSUPPORTED
        with pytest.raises(sf.SflsError) as e:
            srv.submit(addr[0], 1, 0)
        assert e.value.status == sf.SFLS_EINVAL
        assert srv.stats()["in_flight"] == 0
    finally:
        srv.close()
    with pytest.raises(sf.SflsError):
        sf.Server(ctx, max_n=1 << 20)
    with pytest.raises(sf.SflsError):
        sf.Server(ctx, max_n=65536, hbm_bytes=1 << 20)  # no room for one request


def test_request_loop_over_size_class_lanes(ctx):
    """Poisson arrivals into two servers on separate streams; every request is
    served, and each result equals the one the request gets alone."""
    ns = [256, 1024, 256, 4096, 1024, 256, 4096, 1024, 256, 256]
    insts = signals(ns, seed=4)
    y, addr = to_device(insts)
    classes = ((1024, 8), (4096, 4))
    lanes = serving.default_lanes(ctx, sf.default_params(precision=sf.SFLS_MIXED),
                                  size_classes=classes, hbm_bytes=(1 << 30, 1 << 30))
    try:
        rng = np.random.default_rng(5)
        arrivals = np.cumsum(rng.exponential(0.002, len(ns)))
        sizes = np.array(ns, np.int64)
        lane_of = [serving.lane_index(classes, n) for n in ns]
        res, lat, stats = serving.run_stream(lanes, lane_of, arrivals, sizes, lambda i: addr[i])
        assert all(r is not None for r in res) and np.all(np.isfinite(lat)) and np.all(lat > 0)
        for li, lane in enumerate(lanes):
            idx = [i for i in range(len(ns)) if lane_of[i] == li]
            alone = run_alone(lane, [insts[i] for i in idx], [addr[i] for i in idx])
            for a, i in zip(alone, idx):
                a.tag = i
                same(a, res[i])
        summ = serving.summarize(lat, sizes, arrivals, stats["wall_s"])
        print(summ, flush=True)
    finally:
        for s in lanes:
            s.close()


def test_host_and_device_signals_give_the_same_result(ctx):
    """A signal in host memory (copied at submission) and the same signal on
    the device (copied by the next round's admission kernel) are served to the
    same bits."""
    insts = signals([512, 1000, 256], seed=5)
    y, addr = to_device(insts)
    host = [np.ascontiguousarray(i.y.astype(np.complex64)) for i in insts]
    out = []
    for use_host in (False, True):
        srv = sf.Server(ctx, max_n=1024, max_slots=4, hbm_bytes=256 << 20)
        try:
            for k, inst in enumerate(insts):
                ptr = host[k].ctypes.data if use_host else addr[k]
                assert srv.submit(ptr, inst.N, k)
            got = {}
            while len(got) < len(insts):
                srv.step()
                for r in srv.poll():
                    got[r.tag] = r
            out.append([got[k] for k in range(len(insts))])
        finally:
            srv.close()
    for a, b in zip(*out):
        same(a, b)


def test_submit_many_admits_in_order_until_full(ctx):
    """sfls_server_submit_many admits requests in order until the slots run
    out (the rest are left to the caller), and each result is bitwise the one
    the request gets when submitted alone."""
    ns = [256, 700, 1024, 300, 512, 128]
    insts = signals(ns, seed=3)
    y, addr = to_device(insts)
    p = sf.default_params(precision=sf.SFLS_MIXED)
    srv = sf.Server(ctx, max_n=1024, max_slots=4, hbm_bytes=1 << 30, params=p)
    try:
        alone = run_alone(srv, insts, addr)
        tags = np.arange(len(insts), dtype=np.uint64)
        ptrs = np.array(addr, dtype=np.uint64)
        nn = np.array(ns, dtype=np.int64)
        first = srv.submit_many(ptrs, nn, tags)
        assert first == 4  # four slots
        nxt, out = first, {}
        for _ in range(100000):
            srv.step()
            for r in srv.poll():
                out[r.tag] = r
            if nxt < len(insts):
                nxt += srv.submit_many(ptrs[nxt:], nn[nxt:], tags[nxt:])
            if len(out) == len(insts):
                break
        assert srv.submit_many(ptrs[:0], nn[:0], tags[:0]) == 0
        with pytest.raises(sf.SflsError):
            srv.submit_many(ptrs[:1], np.array([1], dtype=np.int64), tags[:1])  # n < 2
    finally:
        srv.close()
    assert sorted(out) == list(range(len(insts)))
    for k in range(len(insts)):
        same(alone[k], out[k])
