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
