"""CPU checks of the benchmark's work accounting (no GPU): the in-sector
matrix-element count used for the H-apply roofline against brute-force
enumeration of the sector."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n,ne,seed", [(6, 3, 1), (7, 3, 2), (8, 4, 3), (9, 5, 4)])
def test_sector_elements_match_enumeration(n, ne, seed):
    import bench
    import paper_2311_01242_amd as vq
    from vqe_inputs import random_integrals
    h0, h, g = random_integrals(n, seed)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    x, _, _ = H.terms()
    na, nb = (ne + 1) // 2, ne // 2

    def in_sector(s):
        return bin(s & 0x55555555).count("1") == na and bin(s & 0xAAAAAAAA).count("1") == nb

    sector = [s for s in range(1 << n) if in_sector(s)]
    # one element per (output, distinct x-mask) with the partner in the sector
    brute = sum(1 for xi in set(int(v) for v in x) for s in sector if in_sector(s ^ xi))
    assert bench.sector_elements(H, n, ne) == brute
    # and the nonzero entries of the sector block of the oracle's dense matrix
    # (random integrals: no element cancels), diagonal included
    if n <= 8:
        from oracle import pauli as P
        m = P.matrix(P.jw_hamiltonian(n, h0, h, g), n)
        assert np.count_nonzero(np.abs(m[np.ix_(sector, sector)]) > 1e-12) == brute


@pytest.mark.parametrize("n,ne", [(6, 3), (8, 4), (9, 4), (10, 5)])
def test_walk_lds_bytes_match_enumeration(n, ne):
    """The beta-pair walk's gather count: (row, alpha pair with one occupied
    orbital, column, beta pair with one occupied orbital), each a coefficient
    and an amplitude; every alpha pair with a beta pair is a group of the
    molecular Hamiltonian (so every such alpha pair is a class)."""
    import itertools
    import bench
    import paper_2311_01242_amd as vq
    from vqe_inputs import random_integrals
    na, nb = (ne + 1) // 2, ne // 2
    oa, ob = (n + 1) // 2, n // 2
    rows = [a for a in range(1 << oa) if bin(a).count("1") == na]
    cols = [b for b in range(1 << ob) if bin(b).count("1") == nb]
    apairs = list(itertools.combinations(range(oa), 2))
    bpairs = list(itertools.combinations(range(ob), 2))
    one = lambda s, p, q: ((s >> p) & 1) != ((s >> q) & 1)
    count = sum(1 for a in rows for p, q in apairs if one(a, p, q)
                for b in cols for r, t in bpairs if one(b, r, t))
    assert bench.walk_lds_bytes(n, ne, 8) == 16 * count
    assert bench.walk_lds_bytes(n, ne, 16) == 24 * count
    # every alpha pair appears with a beta pair among the Hamiltonian's x-masks
    h0, h, g = random_integrals(n, 5)
    x, _, _ = vq.Hamiltonian.from_integrals(n, h0, h, g).terms()
    xa = {sum(((int(v) >> (2 * i)) & 1) << i for i in range(oa)) for v in x
          if bin(sum(((int(v) >> (2 * i + 1)) & 1) << i for i in range(ob))).count("1") == 2}
    assert all((1 << p) | (1 << q) in xa for p, q in apairs)


def test_traffic_reported_only_for_its_workload_and_source(tmp_path, monkeypatch):
    """roofline.traffic comes from the counter file only for the workload it
    was measured on and while the kernel source hash matches."""
    import json
    import bench

    def write(workload, sha):
        rec = {"workload": workload,
               "kernels": {"adjoint": {"bytes_per_launch": 123.0, "source_sha256": sha}}}
        f = tmp_path / "traffic.json"
        f.write_text(json.dumps(rec))
        # key -> (file, the workload the file must name)
        monkeypatch.setattr(bench, "TRAFFIC", {"w1": (str(f), "w1"), "w2": (str(f), "w2")})

    class Batch:   # phase times (ms) and work counters of one evaluation
        S = 1

        def profile(self, theta, reps):
            return [1.0, 1.0, 2.0, 0.1]

        def work(self):
            return np.array([1e9, 0.0, 2e9, 0.0, 10.0, 1.0, 10.0, 0.0])

    def adj_traffic(key):
        r = bench.roofline(Batch(), None, 1, [], [], pairs=1000, traffic_key=key)
        assert r["dominant_phase"] == "adjoint"
        assert r["phases"]["adjoint"]["traffic"] == r["traffic"]
        return r["traffic"]

    sha = bench.source_hash(bench.PHASE_KERNELS["adjoint"][1])
    write("w1", sha)
    assert adj_traffic("w1") == 123.0
    assert adj_traffic("w2") is None
    assert adj_traffic(None) is None
    write("w1", "0" * 64)   # kernel changed since the counters were taken
    assert adj_traffic("w1") is None
