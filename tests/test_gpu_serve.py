"""Serving loop on the GPU: every request served inside a mixed, continuously
batched stream gives the same bytes as the same request served alone, and
both equal the oracle's product of the request's matrix with its inputs."""
import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import serve as SV

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def outputs_of(server, reqs):
    return [[server.arena[r.out_off + j * r.block_bytes: r.out_off + (j + 1) * r.block_bytes].cpu().numpy()
             for j in range(r.n_out)] for r in reqs]


def expected(server, req, pool_h, pool_ptr):
    G = np.array(server.cache.generator(req.n, req.p), dtype=np.uint8)
    ins = [pool_h[x - pool_ptr: x - pool_ptr + req.block_bytes] for x in req.inputs]
    if req.erased:
        D, surv = oracle.decode_matrix(G, req.n, req.p, list(req.erased))
        assert surv == server.cache.get(req.n, req.p, req.erased).in_blocks
    else:
        D = G[req.n:]
    return oracle.apply(D, [np.ascontiguousarray(b) for b in ins])


def test_mix_equals_alone_equals_oracle():
    pool_bytes = 8 << 20
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    pool = torch.randint(0, 256, (pool_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    pool_h = pool.cpu().numpy()
    reqs = SV.make_requests(0.004, 20000.0, seed=5, pool_ptr=pool.data_ptr(), pool_bytes=pool_bytes,
                            hi=1 << 20)
    assert len(reqs) > 40
    # A budget far below the total forces admission back-pressure and many
    # batches in flight; small batches interleave codecs and sizes.
    server = SV.Server(generator_fn=oracle.cauchy, budget_bytes=16 << 20, n_slots=3, max_batch=7, warm=False)
    for r in reqs:
        server.cache.get(r.n, r.p, r.erased)
    for r in reqs:
        r.arrival = 0.0
    mixed = {}

    def grab(done):
        mixed.update({r.rid: o for r, o in zip(done, outputs_of(server, done))})
    server.serve(reqs, realtime=False, on_done=grab)
    torch.cuda.synchronize()
    assert all(r.done >= 0 for r in reqs) and len(mixed) == len(reqs)
    assert server.batches >= len(reqs) // 7
    assert len({r.out_off for r in reqs}) > 1  # the arena's space was reused across batches
    mixed = [mixed[r.rid] for r in reqs]
    alone = []
    for r in reqs:
        server.serve([r], realtime=False)
        torch.cuda.synchronize()
        alone += outputs_of(server, [r])
    for k, r in enumerate(reqs):
        for j in range(r.n_out):
            assert np.array_equal(mixed[k][j], alone[k][j]), "request %d output %d" % (k, j)
    for k in range(0, len(reqs), 5):
        want = expected(server, reqs[k], pool_h, pool.data_ptr())
        for j in range(reqs[k].n_out):
            assert np.array_equal(alone[k][j], want[j]), "oracle: request %d output %d" % (k, j)


def test_native_loop_realtime_and_argument_errors():
    """The library's loop on a short Poisson stream in real time: every
    request completes after its arrival and equals the oracle; requests out
    of arrival order, with an input inside the output arena or larger than
    the budget are refused before any launch."""
    pool_bytes = 8 << 20
    g = torch.Generator(device="cuda")
    g.manual_seed(12)
    pool = torch.randint(0, 256, (pool_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    pool_h = pool.cpu().numpy()
    reqs = SV.make_requests(0.01, 20000.0, seed=6, pool_ptr=pool.data_ptr(), pool_bytes=pool_bytes, hi=1 << 20)
    server = SV.Server(generator_fn=oracle.cauchy, budget_bytes=64 << 20, n_slots=4, max_batch=16, warm=False)
    got = {}

    def grab(done):
        got.update({r.rid: o for r, o in zip(done, outputs_of(server, done))})
    wall = server.serve(reqs, on_done=grab)
    torch.cuda.synchronize()
    assert len(got) == len(reqs) and wall >= reqs[-1].arrival
    assert all(r.done >= r.arrival for r in reqs)
    for k in range(0, len(reqs), 7):
        want = expected(server, reqs[k], pool_h, pool.data_ptr())
        for j in range(reqs[k].n_out):
            assert np.array_equal(got[reqs[k].rid][j], want[j]), "request %d output %d" % (k, j)
    from paper_2108_02692_amd import EcError
    a, b = reqs[0], reqs[1]
    a.arrival, b.arrival = 0.002, 0.001
    with pytest.raises(EcError) as e:
        server.serve([a, b])  # arrivals out of order
    assert e.value.name == "EC_ERR_ARG"
    inside = SV.Request(0, 0.0, a.n, a.p, a.erased, a.block_bytes, inputs=[server.base] + a.inputs[1:])
    with pytest.raises(EcError) as e:
        server.serve([inside])  # an input inside the output arena
    assert e.value.name == "EC_ERR_ARG"
    small = SV.Server(generator_fn=oracle.cauchy, budget_bytes=256 << 10, n_slots=2, max_batch=4, warm=False)
    big = max(reqs, key=lambda r: r.bytes)
    big.arrival = 0.0
    assert big.bytes > 256 << 10
    with pytest.raises(EcError) as e:
        small.serve([big])
    assert e.value.name == "EC_ERR_CAPACITY"


def test_native_loop_mixed_slot_budgets():
    """Requests whose programs use different slot budgets (one kernel
    instance per launch) interleaved in one run, all present at once: the
    loop splits its batches at each change of budget, warms each budget's
    kernels, and every output equals the oracle."""
    import paper_2108_02692_amd as E
    rng = np.random.default_rng(21)
    pool_bytes = 4 << 20
    pool_h = rng.integers(0, 256, pool_bytes, dtype=np.uint8)
    pool = torch.from_numpy(pool_h).cuda()
    arena = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    codecs = [(10, 4, (), 38), (4, 2, (), 24), (6, 3, (1, 7), 32), (10, 4, (2, 4, 5, 11), 38)]
    progs = {c: E.ec_compile_slp(c[0], c[1], oracle.cauchy(c[0], c[1]).tolist(), list(c[2]), slot_budget=c[3])
             for c in codecs}
    reqs, meta = [], []
    for k in range(40):
        c = codecs[k % len(codecs)] if k % 5 else codecs[1]
        prog = progs[c]
        bb = 512 * int(rng.integers(1, 80))
        offs = (rng.integers(0, (pool_bytes - bb) // 512, len(prog.in_blocks)) * 512).tolist()
        reqs.append((0.0, prog, [pool.data_ptr() + o for o in offs], bb))
        meta.append((c, offs, bb))
    srv = E.ec_server_create(arena, arena.numel(), budget_bytes=16 << 20, n_slots=3, max_batch=8)
    got = {}

    def grab(ids, out_offs):
        for i, off in zip(ids, out_offs):
            c, _, bb = meta[i]
            got[i] = arena[off: off + len(progs[c].out_blocks) * bb].cpu().numpy().copy()
    done, offs, wall, nb = srv.run(reqs, realtime=False, on_done=grab)
    torch.cuda.synchronize()
    assert len(got) == len(reqs) and all(t >= 0 for t in done) and nb >= 10
    for i, (c, ins, bb) in enumerate(meta):
        n, p, er, _ = c
        G = oracle.cauchy(n, p)
        data = [pool_h[o: o + bb] for o in ins]
        if er:
            D, surv = oracle.decode_matrix(G, n, p, list(er))
            assert surv == progs[c].in_blocks
        else:
            D = G[n:]
        want = np.concatenate(oracle.apply(D, [np.ascontiguousarray(b) for b in data]))
        assert np.array_equal(got[i], want), "request %d %s" % (i, c)
    srv.free()


def test_native_encodes_in_the_loop():
    """A server whose encode programs have native kernels: requests served
    alone run them, batched ones the interpreter; every output equals the
    oracle."""
    pool_bytes = 8 << 20
    g = torch.Generator(device="cuda")
    g.manual_seed(14)
    pool = torch.randint(0, 256, (pool_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    pool_h = pool.cpu().numpy()
    server = SV.Server(generator_fn=oracle.cauchy, budget_bytes=64 << 20, n_slots=4, max_batch=16, warm=False,
                       native_encodes=True)
    for n, p in ((10, 4), (6, 3)):
        assert server.cache.get(n, p).info["native"] == E.NATIVE_WHOLE | E.NATIVE_PAIRS | E.NATIVE_BLOCKS
        assert server.cache.get(n, p, (1,)).info["native"] == 0
    reqs = SV.make_requests(0.01, 20000.0, seed=9, pool_ptr=pool.data_ptr(), pool_bytes=pool_bytes, hi=1 << 20)
    assert any(not r.erased for r in reqs) and any(r.erased for r in reqs)
    got = {}

    def grab(done):
        got.update({r.rid: o for r, o in zip(done, outputs_of(server, done))})
    server.serve(reqs, on_done=grab)
    torch.cuda.synchronize()
    for r in [r for r in reqs if not r.erased] + reqs[::5]:
        want = expected(server, r, pool_h, pool.data_ptr())
        for j in range(r.n_out):
            assert np.array_equal(got[r.rid][j], want[j]), "request %d output %d" % (r.rid, j)
    # the same requests all at once: batches of several requests
    got.clear()
    for r in reqs:
        r.arrival = 0.0
    server.serve(reqs, realtime=False, on_done=grab)
    torch.cuda.synchronize()
    for r in reqs[::3]:
        want = expected(server, r, pool_h, pool.data_ptr())
        for j in range(r.n_out):
            assert np.array_equal(got[r.rid][j], want[j]), "drain: request %d output %d" % (r.rid, j)
