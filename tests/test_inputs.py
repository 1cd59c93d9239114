"""Module-I inputs in the paper's conventions (App. G) mapped onto requests."""
import numpy as np
import pytest

from paper_2105_13611_amd import inputs, workload as W

# an input in the module-I keyword format (values made up for the test)
EXAMPLE = """molecules off
print 1
velocities values 4 0.0 1.0 2.5 4.0
odf number 3
user defined binning on
odf mean arithmetic
abundance scale   0.5 abundance change 1 0.92000 2 0.07800
 abundance change  6  -3.50  8  -3.20 26  -4.60
 abundance change 12  -4.40
begin
end
"""


def test_keywords():
    inp = inputs.parse_odf_input(EXAMPLE)
    assert inp.vturbs_kms == [0.0, 1.0, 2.5, 4.0]
    assert inp.mean == "arithmetic"
    assert inp.abundance_scale == 0.5
    assert inp.abundance_change == {1: 0.92, 2: 0.078, 6: -3.5, 8: -3.2, 26: -4.6, 12: -4.4}
    # the defaults of a run without the keywords
    bare = inputs.parse_odf_input("print 1\n")
    assert bare.vturbs_kms == [0.0] and bare.mean == "geometric" and bare.abundance_scale == 1.0
    with pytest.raises(ValueError):
        inputs.parse_odf_input("velocities values 3 0.0 1.0\n")


def test_abundances_relative_to_hydrogen():
    inp = inputs.parse_odf_input(EXAMPLE)
    a = inputs.abundances_relative_to_h(inp, [2, 6, 12, 26])
    np.testing.assert_allclose(a, [0.078 / 0.92, 0.5 * 10 ** -3.5 / 0.92, 0.5 * 10 ** -4.4 / 0.92,
                                   0.5 * 10 ** -4.6 / 0.92], rtol=1e-15)
    # round trip from abundances relative to H
    rng = np.random.default_rng(1)
    A = 10.0 ** rng.uniform(-12, -4, 5)
    x_h = 0.9
    text = "abundance scale 1.0 abundance change 1 0.9\n" + "".join(
        f" abundance change {z} {np.log10(A[k] * x_h):.15f}\n" for k, z in enumerate(range(3, 8)))
    back = inputs.abundances_relative_to_h(inputs.parse_odf_input(text), range(3, 8))
    np.testing.assert_allclose(back, A, rtol=1e-12)
    with pytest.raises(ValueError):
        inputs.abundances_relative_to_h(inp, [7])          # no entry for N


def test_tpgrid_expansion_matches_the_table_order():
    g = W.dfsynthe_tp_grid((0.0, 2.0))
    T = 2000.0 * 100.0 ** (np.arange(57) / 56.0)
    lp = -4.0 + 0.5 * np.arange(25)
    text = "57\n25\n" + "".join(f"{float(t)!r}\n" for t in T) + "".join(f"{float(p)!r}\n" for p in lp)
    pts = inputs.parse_tpgrid(text, [0.0, 2.0])
    assert pts.n_points == 2 * 57 * 25
    np.testing.assert_array_equal(pts.T_K, g.T_K)
    np.testing.assert_array_equal(pts.log10_P, g.log10_P)
    np.testing.assert_array_equal(pts.vturb_kms, g.vturb_kms)
    lin = inputs.parse_tpgrid("1\n2\n5000.0\n1.0e4\n1.0e2\n", [1.5], log_pressure=False)
    np.testing.assert_allclose(lin.log10_P, [4.0, 2.0])
    with pytest.raises(ValueError):
        inputs.parse_tpgrid("2\n2\n5000.0\n1.0\n", [0.0])
