"""Host-side logic of the Sec. 7.3 experiment runner (no GPU)."""
import numpy as np

import oracle as O


def test_partition_pieces_split_at_boundaries():
    # the per-partition piece offsets partition the pieces exactly at the domain ends (host logic)
    from paper_2401_00109_amd import experiments as E
    x = E.noise_series(1000)
    so = np.array([0, 1000], np.int64)
    for D in (1, 7, 100, 999):
        ln, ic, po = O.compress(x, so, D, 0.3)
        values, dso, dpo, t0 = E._domains(x, ln, D)
        assert dpo[0] == 0 and dpo[-1] == ln.size
        for d in range(dpo.size - 1):
            assert ln[dpo[d]:dpo[d + 1]].sum() == dso[d + 1] - dso[d] - 1
