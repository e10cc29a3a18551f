"""Symbolic simulator of the executor's device bytecode (test helper).

Written from the block format documented in ``csrc/bytecode.hpp``, not from
the emitter: it walks the blocks as the device does, tracks every slot's
value as a set of input strips (the set semantics of Sec. 4.1), and models
the in-order vector-memory counter, so it reports a read of a slot whose
load may still be in flight, a register write racing a load, or a wrong
output.  Returns {output strip: value bitset}.
"""


class SimError(AssertionError):
    pass


def simulate(words, slots, n_in_strips, n_out_strips, max_vmcnt=63):
    val = {}          # slot -> bitset value
    pending = {}      # slot -> vm sequence of the load filling it
    issued = 0        # vector memory ops issued so far
    done_upto = -1    # every op with sequence <= done_upto has completed
    acc = 0
    out = {}
    pc = 0
    steps = 0

    def complete(seq_limit):
        nonlocal done_upto
        done_upto = max(done_upto, seq_limit)

    def ready(s):
        return pending.get(s, -1) <= done_upto

    while True:
        steps += 1
        if steps > 1_000_000:
            raise SimError("no HALT")
        if pc + 16 > len(words):
            raise SimError("block window runs past the program at %d" % pc)
        h0, h1 = words[pc], words[pc + 1]
        n = h0 & 15
        if n > 14:
            raise SimError("too many operands")
        if h0 & (1 << 4):  # LD
            s, c = (h0 >> 5) & 63, (h0 >> 11) & 0x7FF
            if s >= slots or c >= n_in_strips:
                raise SimError("LD out of range")
            if not ready(s):
                raise SimError("LD into slot %d while its previous load is in flight" % s)
            val[s] = 1 << c
            pending[s] = issued
            issued += 1
            if issued - 1 - done_upto > max_vmcnt + 1:
                raise SimError("more vector memory ops outstanding than the counter holds")
        if h0 & (1 << 22):  # WAIT
            cnt = (h0 >> 23) & 63
            complete(issued - 1 - cnt)
        for k in range(n):
            o = words[pc + 2 + k]
            if o & 3 or o >> 8:
                raise SimError("bad operand word")
            s = o >> 2
            if s >= slots:
                raise SimError("operand slot out of range")
            if s not in val:
                raise SimError("read of never-written slot %d" % s)
            if not ready(s):
                raise SimError("read of slot %d before its load completed" % s)
            acc ^= val[s]
        if h1 & 1:  # PUT
            s = (h1 >> 5) & 63
            if s >= slots:
                raise SimError("PUT out of range")
            if not ready(s):
                raise SimError("PUT into slot %d while a load into it is in flight" % s)
            val[s] = acc
            pending.pop(s, None)
        if h1 & 2:  # STORE
            o = (h1 >> 11) & 0x7FF
            if o >= n_out_strips:
                raise SimError("STORE out of range")
            out[o] = acc
            issued += 1
        if h1 & 4:  # CLEAR
            acc = 0
        pc += 2 + n
        if h1 & 8:  # HALT
            break
    if acc != 0:
        raise SimError("accumulator not cleared at HALT")
    return out
