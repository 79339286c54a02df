"""CPU checks of the benchmark's work accounting (no GPU): the in-sector
(output, term) pair count used for the H-apply roofline against brute-force
enumeration of the sector."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n,ne,seed", [(6, 3, 1), (7, 3, 2), (8, 4, 3), (9, 5, 4)])
def test_sector_pairs_match_enumeration(n, ne, seed):
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
    brute = sum(1 for xi in x for s in sector if in_sector(s ^ int(xi)))
    assert bench.sector_pairs(H, n, ne) == brute
