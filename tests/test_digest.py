"""The population digest (an output for comparing whole populations, not
part of the method): the oracle's definition written out once more, and the
properties the comparison relies on."""
import numpy as np

import oracle


def _d(L=8, q=5, seed=2**40 + 3):
    return oracle.Desc(L, q, 10, np.array([0.0, 0.5]), 1, seed)


def test_digest_definition():
    """Sum over slots k and dwords n of (Philox(n, k, i, 5 << 28) as 64 bits
    | 1) * (spins 4n..4n+3 packed little endian), modulo 2^64."""
    d = _d()
    rng = np.random.default_rng(1)
    spins = rng.integers(0, 5, size=(3, 64), dtype=np.uint8)
    key = [d.seed & 0xFFFFFFFF, d.seed >> 32]
    want = 0
    for k in range(3):
        for n in range(16):
            w = oracle.philox([n, k, 7, 5 << 28], key)
            r = ((int(w[1]) << 32) | int(w[0])) | 1
            dw = int.from_bytes(bytes(spins[k, 4 * n:4 * n + 4]), "little")
            want = (want + r * dw) % 2**64
    assert oracle.digest(d, 7, spins) == want


def test_digest_properties():
    """Zero population -> 0; linear in the dwords slot by slot; any single
    changed spin changes it; the step index and the slot order matter."""
    d = _d()
    rng = np.random.default_rng(2)
    a = rng.integers(0, 5, size=(2, 64), dtype=np.uint8)
    z = np.zeros_like(a)
    assert oracle.digest(d, 3, z) == 0
    a0, a1 = a.copy(), a.copy()
    a0[1] = 0
    a1[0] = 0
    assert oracle.digest(d, 3, a) == (oracle.digest(d, 3, a0) + oracle.digest(d, 3, a1)) % 2**64
    base = oracle.digest(d, 3, a)
    for _ in range(50):
        b = a.copy()
        k, s = rng.integers(0, 2), rng.integers(0, 64)
        b[k, s] = (b[k, s] + rng.integers(1, 5)) % 5
        assert oracle.digest(d, 3, b) != base
    assert oracle.digest(d, 4, a) != base
    assert oracle.digest(d, 3, a[::-1].copy()) != base


def test_run_reports_the_digest_of_its_populations():
    d = oracle.Desc(8, 4, 50, np.array([0.0, 0.4, 0.8]), 2, 9, resample=oracle.RESAMPLE_MULTINOMIAL)
    o = oracle.run(d, digest=True, final=True)
    assert o["digest"][-1] == oracle.digest(d, 2, o["final_spins"])
