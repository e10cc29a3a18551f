"""The device program pool: programs uploaded together take one device
allocation at most, identical records are stored once, the space of freed
programs is reused, and programs placed in the pool still give the oracle's
results (decodes of every erasure pattern of a small codec)."""
import ctypes
import gc

import numpy as np
import pytest

import oracle
import paper_2108_02692_amd as E
from paper_2108_02692_amd import batching as B

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, P = 7, 3  # 176 programs: the encode and every pattern of 1..3 erasures


def compiled(keys):
    cache = B.ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=38, generator_fn=oracle.cauchy)
    cache.warm(keys)
    return cache


def test_upload_many_one_allocation_sharing_and_reuse():
    torch.zeros(1, device="cuda")
    gc.collect()  # programs other tests left behind go now, not mid-test
    keys = [(N, P, er) for er in B.ProgramCache(level=E.LEVEL_PLAIN, slots=38).all_patterns(N, P)]
    assert len(keys) == 176
    c0, i0, b0 = E.ec_program_pool_stats()
    first = compiled(keys)
    first.upload()
    c1, i1, b1 = E.ec_program_pool_stats()
    assert c1 - c0 <= 1, "one upload of %d programs took %d allocations" % (len(keys), c1 - c0)
    assert 0 < i1 - i0 <= len(keys)
    assert b1 > b0 and b1 % 256 == 0

    # the same programs compiled again: stored once, nothing allocated
    second = compiled(keys)
    second.upload()
    assert E.ec_program_pool_stats() == (c1, i1, b1)

    # the records in the pool decode as the oracle does, for every pattern
    G = oracle.cauchy(N, P)
    rng = np.random.default_rng(3)
    bb = 8192
    data = [rng.integers(0, 256, bb, dtype=np.uint8) for _ in range(N)]
    blocks = data + oracle.encode(G, N, P, data)
    dev = [torch.from_numpy(b).cuda() for b in blocks]
    for er in [k[2] for k in keys if k[2]]:
        prog = second.get(N, P, er)
        outs = [torch.empty(bb, dtype=torch.uint8, device="cuda") for _ in er]
        E.ec_decode(prog, [dev[i] for i in prog.in_blocks], outs, bb)
        torch.cuda.synchronize()
        for e, o in zip(er, outs):
            assert np.array_equal(o.cpu().numpy(), blocks[e]), "erased %s block %d" % (er, e)

    # freed programs give their space back; a new set fits in it
    del first, second, prog
    gc.collect()
    assert E.ec_program_pool_stats() == (c1, i0, b0)
    third = compiled(keys)
    third.upload()
    assert E.ec_program_pool_stats() == (c1, i1, b1)
    del third
    gc.collect()


def test_upload_many_argument_errors():
    torch.zeros(1, device="cuda")
    from paper_2108_02692_amd import EcError
    E.ec_program_upload_many([])  # nothing to do
    for arr, n in [(None, 1), ((ctypes.c_void_p * 2)(None, None), 2), ((ctypes.c_void_p * 1)(None), -1)]:
        with pytest.raises(EcError) as e:
            E._check(E.lib().ec_program_upload_many(arr, n), "ec_program_upload_many")
        assert e.value.name == "EC_ERR_ARG"
