"""Independent simulator of the executor's record stream (written from the
format described in csrc/bytecode.hpp, sharing no code with the library).

Slots hold values under the set semantics of Sec. 4.1 (a Python int whose bit
c stands for input strip c).  The vector memory counter is modelled exactly:
a load lands only when a WAIT retires it (in issue order, stores included),
so reading or accumulating into a slot whose load may still be in flight is
an error, as is loading into such a slot.  The program is run for several
consecutive tiles from all-zero slots, each tile starting from the state the
previous one left, and every tile must store the same values and leave
every slot zero (the next tile may run another program).
"""

KINDS = {0: "RUN", 1: "INPUT", 2: "INPUT_LD", 3: "VALUE", 4: "STORE", 5: "LOAD", 6: "HALT", 7: "PREFETCH"}


class SimError(AssertionError):
    pass


def fields(h0, h1):
    return {
        "pull4": h0 & 0xFF, "b8": (h0 >> 8) & 1, "kind": (h0 >> 9) & 7, "bytes": (h0 >> 12) & 0x7F,
        "runoff": (h0 >> 19) & 0x1FF, "h0_hi": h0 >> 28,
        "wait8": h1 & 0x1FF, "ld16": (h1 >> 9) & 0x3FF, "blk": (h1 >> 19) & 0x1F, "j": (h1 >> 24) & 7,
        "h1_hi": h1 >> 27,
    }


def check(cond, msg):
    if not cond:
        raise SimError(msg)


def simulate(words, slots, n_in_blocks, n_out_blocks, tiles=2):
    """Returns {output strip index: value} (identical for every tile)."""
    val = [0] * slots
    busy = [False] * slots
    first = None
    for _ in range(tiles):
        vm = []
        out = {}
        acc = 0
        pc = 0
        while True:
            check(pc + 16 <= len(words), "window past the end at %d" % pc)
            f = fields(words[pc], words[pc + 1])
            kind = KINDS.get(f["kind"])
            check(kind is not None, "bad kind at %d" % pc)
            if kind == "HALT":
                check(words[pc] >> 12 & 0x7F == 8 and words[pc + 1] == 0, "HALT fields")
                check(all(w == 0 for w in words[pc + 2:]), "words after HALT")
                check(len(words) - pc >= 18, "no zero window after HALT")
                break
            check(f["b8"] == 0 and f["h0_hi"] == 0 and f["h1_hi"] == 0, "reserved bits at %d" % pc)
            nb = f["bytes"]
            check(nb >= 8 and nb % 4 == 0 and nb <= 64, "record size at %d" % pc)
            n = (nb - 8) // 4
            check(f["runoff"] == (14 - n) * 20, "run entry at %d" % pc)
            check(f["pull4"] % 4 == 0, "pull field")
            pull = f["pull4"] // 4
            pulls = kind in ("INPUT", "INPUT_LD", "VALUE", "STORE")
            loads = kind in ("INPUT_LD", "LOAD")
            waits = kind in ("INPUT", "INPUT_LD")
            check(pulls or pull == 0, "stray pull field at %d" % pc)
            check(waits or f["wait8"] == 0, "stray wait at %d" % pc)
            check(f["wait8"] % 8 == 0 and f["ld16"] % 16 == 0, "scaled fields at %d" % pc)
            check(loads or f["ld16"] == 0, "stray load slot at %d" % pc)
            check(loads or kind in ("STORE", "PREFETCH") or (f["blk"] == 0 and f["j"] == 0),
                  "stray strip at %d" % pc)
            if waits:
                keep = f["wait8"] // 8
                while len(vm) > keep:
                    s = vm.pop(0)
                    if s is not None:
                        busy[s] = False
            if pulls:
                check(pull < slots, "pull slot range")
                check(not busy[pull], "pull of slot %d before its load landed (pc %d)" % (pull, pc))
                acc = val[pull]
            if loads:
                s = f["ld16"] // 16
                check(s < slots and f["blk"] < n_in_blocks, "load fields at %d" % pc)
                check(not busy[s], "load into slot %d with a load in flight" % s)
                val[s] = 1 << (8 * f["blk"] + f["j"])
                busy[s] = True
                vm.append(s)
            if kind == "PREFETCH":
                check(f["blk"] < n_in_blocks and n == 0, "prefetch fields at %d" % pc)
                vm.append(None)
            if kind == "STORE":
                check(n_in_blocks <= f["blk"] < n_in_blocks + n_out_blocks, "store block at %d" % pc)
                o = 8 * (f["blk"] - n_in_blocks) + f["j"]
                check(o not in out, "strip %d stored twice" % o)
                out[o] = acc
                vm.append(None)
            for q in range(n):
                w = words[pc + 2 + q]
                check(w % 4 == 0 and w // 4 < slots, "operand at %d" % pc)
                s = w // 4
                check(not busy[s], "XOR into slot %d with a load in flight" % s)
                val[s] ^= acc
            pc += 2 + n
        check(not any(busy), "load left unconsumed")
        check(not any(val), "a slot is not zero at the end of the tile")
        if first is None:
            first = out
        else:
            check(out == first, "a later tile stored different values")
    return first
