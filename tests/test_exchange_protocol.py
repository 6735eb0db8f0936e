"""The exchange solve's synchronisation protocol (paper_2511_11514_amd/csrc/mesh.hip),
checked on the CPU by running it under random interleavings of its blocks.

Model: G blocks; block b owns rows of x (its f and p) and rows of y (its g and q).
Potentials travel as words (version, value) in two buffers per potential, the word
of version v in buffer v mod 2.  A block publishes its own rows' g, p and q at
version 0, then per iteration k:
    half 0: gather g and p of every row at version k; publish its f and p at k + 1;
    half 1: gather f at version k + 1 and q at version k; publish its g and q at k + 1.
A gather reads each word until it carries the awaited version (any order, any
number of retries).  The properties: a read never finds a word of a later version
than the one it awaits (no word is overwritten before every reader has taken
it), and every interleaving runs to completion (no deadlock).  A planted mistake
(one buffer instead of two) must break the first property."""
import random

import pytest


def _run(G, rows, K, buffers, seed):
    """One random interleaving; returns None or a description of the first violation."""
    rng = random.Random(seed)
    kinds = ("f", "g", "p", "q")
    n = {k: rows * G for k in kinds}
    own = {b: list(range(b * rows, (b + 1) * rows)) for b in range(G)}
    mem = {k: [[(-1, None)] * n[k] for _ in range(buffers)] for k in kinds}

    def program(b):
        # the block's actions in order: ("pub", kind, row, version) or ("get", [(kind, version)])
        acts = [("pub", k, r, 0) for k in ("g", "p", "q") for r in own[b]]
        for k in range(K):
            acts.append(("get", [("g", k), ("p", k)]))
            acts += [("pub", kd, r, k + 1) for kd in ("f", "p") for r in own[b]]
            acts.append(("get", [("f", k + 1), ("q", k)]))
            acts += [("pub", kd, r, k + 1) for kd in ("g", "q") for r in own[b]]
        return acts

    progs = {b: program(b) for b in range(G)}
    pc = {b: 0 for b in range(G)}
    pending = {b: None for b in range(G)}
    while True:
        live = [b for b in range(G) if pc[b] < len(progs[b])]
        if not live:
            return None
        ready = []
        for b in live:
            act = progs[b][pc[b]]
            if act[0] == "pub":
                ready.append(b)
                continue
            if pending[b] is None:
                pending[b] = [(kd, v, i) for kd, v in act[1] for i in range(n[kd])]
                rng.shuffle(pending[b])
            for kd, v, i in pending[b]:
                ver, _ = mem[kd][v % buffers][i]
                if ver > v:
                    return f"block {b} awaited {kd}[{i}] version {v}, found {ver}"
            if any(mem[kd][v % buffers][i][0] == v for kd, v, i in pending[b]):
                ready.append(b)
        if not ready:
            return "deadlock"
        b = rng.choice(ready)
        act = progs[b][pc[b]]
        if act[0] == "pub":
            _, kd, r, v = act
            mem[kd][v % buffers][r] = (v, (b, v))
            pc[b] += 1
        else:
            # take one word that has arrived (a read of a word not yet there is a retry)
            arrived = [w for w in pending[b] if mem[w[0]][w[1] % buffers][w[2]][0] == w[1]]
            pending[b].remove(rng.choice(arrived))
            if not pending[b]:
                pending[b] = None
                pc[b] += 1


@pytest.mark.parametrize("G,rows,K", [(2, 1, 4), (3, 2, 5), (4, 1, 6)])
def test_two_buffers_never_overwrite_an_awaited_word_and_never_deadlock(G, rows, K):
    for seed in range(300):
        assert _run(G, rows, K, buffers=2, seed=seed) is None, seed


def test_one_buffer_overwrites_an_awaited_word():
    """Planted mistake: with one buffer a fast block's next version replaces a word
    a slow block still awaits, which some interleaving exposes."""
    found = [_run(3, 1, 5, buffers=1, seed=s) for s in range(300)]
    assert any(f is not None and "found" in f for f in found)
