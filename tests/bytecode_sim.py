"""Symbolic simulator of the executor's device bytecode (test helper).

Written from the block format documented in ``csrc/bytecode.hpp``, not from
the emitter: it walks the 16-word blocks as the device does, tracks every
slot's value as a set of input strips (the set semantics of Sec. 4.1), and
models the in-order vector-memory counter, so it reports a read of a slot
whose load may still be in flight, a register write racing a load, an
uninitialised read, or a wrong output.  Returns {output strip: bitset}.
"""

BLOCK = 16


class SimError(AssertionError):
    pass


def simulate(words, slots, n_in_strips, n_out_strips, max_vmcnt=63):
    if len(words) % BLOCK:
        raise SimError("program is not a whole number of blocks")
    val = {}          # slot -> bitset value
    pending = {}      # slot -> vm sequence of the load filling it
    issued = 0
    done_upto = -1
    acc = 0
    out = {}
    pc = 0

    def ready(s):
        return pending.get(s, -1) <= done_upto

    def check_slot(s, what):
        if s >= slots:
            raise SimError("%s slot %d out of range" % (what, s))

    def read(s):
        if s not in val:
            raise SimError("read of never-written slot %d" % s)
        if not ready(s):
            raise SimError("read of slot %d before its load completed" % s)
        return val[s]

    def write(s):
        if not ready(s):
            raise SimError("write to slot %d while a load into it is in flight" % s)
        pending.pop(s, None)

    while True:
        if pc + 2 * BLOCK > len(words):
            raise SimError("block at %d has no read-ahead block after it" % pc)
        h0, h1 = words[pc], words[pc + 1]
        np_, nq = h0 & 15, (h0 >> 4) & 15
        if np_ + nq > 14:
            raise SimError("too many operands")
        ops = words[pc + 2: pc + BLOCK]
        for k, o in enumerate(ops):
            used = k < np_ or k >= 14 - nq
            if (o & 3 or o >> 8) and used:
                raise SimError("bad operand word")
            if not used and o:
                raise SimError("unused operand word is not zero")
        if h0 & (1 << 8):  # LD
            s, c = (h0 >> 9) & 63, (h0 >> 15) & 0x7FF
            check_slot(s, "LD")
            if c >= n_in_strips:
                raise SimError("LD strip out of range")
            if not ready(s):
                raise SimError("LD into slot %d while its previous load is in flight" % s)
            val[s] = 1 << c
            pending[s] = issued
            issued += 1
            if issued - 1 - done_upto > max_vmcnt + 1:
                raise SimError("more vector memory ops outstanding than the counter holds")
        if h0 & (1 << 26):  # WAIT
            done_upto = max(done_upto, issued - 1 - (h1 & 63))
        for k in range(np_):  # PULL
            s = ops[k] >> 2
            check_slot(s, "PULL")
            acc ^= read(s)
        if h1 & (1 << 6):  # PUT
            s = (h1 >> 7) & 63
            check_slot(s, "PUT")
            write(s)
            val[s] = acc
        if h1 & (1 << 13):  # STORE
            o = (h1 >> 14) & 0x7FF
            if o >= n_out_strips:
                raise SimError("STORE out of range")
            out[o] = acc
            issued += 1
        for k in range(14 - nq, 14):  # PUSH / PUSHSET
            s = ops[k] >> 2
            check_slot(s, "PUSH")
            if h0 & (1 << 27):
                write(s)
                val[s] = acc
            else:
                cur = read(s)
                write(s)
                val[s] = cur ^ acc
        if h1 & (1 << 25):
            acc = 0
        if h0 >> 28 or h1 >> 27:
            raise SimError("reserved header bits set")
        pc += BLOCK
        if h1 & (1 << 26):  # HALT
            break
    if acc != 0:
        raise SimError("accumulator not cleared at HALT")
    if pc + BLOCK != len(words):
        raise SimError("words after the read-ahead block")
    return out
