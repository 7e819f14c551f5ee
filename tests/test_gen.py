"""Synthetic inputs: determinism, sizes and the paper's schedule identity."""
import numpy as np

from paper_2603_22274_amd import gen


def test_configs_deterministic_and_sized():
    a, b = gen.config0(), gen.config0()
    assert a.digest() == b.digest()
    assert a.n_atoms == 668 and a.n_windows == 12 and len(a.waters) == 216
    c = gen.config1()
    assert c.n_atoms == 7540 and c.n_windows == 20 and len(c.waters) == 2500
    assert abs(c.ewald_alpha - 0.262826) < 1e-6 and abs(a.ewald_alpha - 0.292029) < 1e-6
    assert abs(float(c.charge.astype(np.float64).sum())) < 1e-5


def test_paper_schedule_window_counts():
    # 29 charge + 45 vdW values share one boundary state (73 windows); the
    # complex leg adds 8 restraint values sharing a second boundary (80).
    assert len(gen.schedule('paper_solvent')) == 73
    assert len(gen.schedule('paper_complex')) == 80
    s = gen.schedule('cfg2')
    assert len(s) == 42 and tuple(s[0]) == (1.0, 1.0, 0.0) and tuple(s[-1]) == (0.0, 0.0, 1.0)


def test_small_complex_restraint_and_excl():
    s = gen.small_complex()
    assert s.restraint_atoms is not None and len(set(s.restraint_atoms.tolist())) == 6
    assert np.all(s.excl[:, 0] < s.excl[:, 1])
    ptr, idx = s.excl_csr()
    assert ptr[-1] == 2 * len(s.excl)
