"""The paper's input and output file formats (host side, no GPU)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2104_03573_amd import paper_io as P


def _box_case(two_clocks=False):
    """A bounded box the paper's files can describe: isothermal walls at z = 0, L, periodic x and
    y, one detector region refined once (2 x 2 x 2 cells)."""
    L = 1e-7
    w = W.gray_slab(N=3000)
    if two_clocks:
        w = W.bulk_gradient(N=3000, modes=W.silicon_like_modes(300.0, impurity_clock=True))
        w["problem"]["n_scat_max"] = 4
    w["geometry"] = {"L": (L, L, L), "unbounded": (False, False, False),
                     "faces": {1: (W.PERIODIC, 0.0, L, 0.0), 3: (W.PERIODIC, 0.0, -L, 0.0),
                               2: (W.PERIODIC, -L, 0.0, 0.0), 4: (W.PERIODIC, L, 0.0, 0.0),
                               5: (W.ISOTHERMAL, 301.0, 0.0, 0.0), 6: (W.ISOTHERMAL, 299.0, 0.0, 0.0)},
                     "cylinders": [], "gradT": (0.0, 0.0, 0.0), "volume": L ** 3}
    w["detectors"] = {"lo": (0.0, 0.0, 0.0), "hi": (L, L, L), "n": (2, 2, 2), "mask": 15}
    return w


@pytest.mark.parametrize("two_clocks", [False, True])
def test_case_round_trip_gives_the_same_run(tmp_path, two_clocks):
    w = _box_case(two_clocks)
    P.write_case(w, str(tmp_path))
    r = P.read_case(str(tmp_path), fmt=w["problem"]["format"], seed=w["seed"],
                    score_axis=w["problem"]["score_axis"])
    assert np.array_equal(r["modes"][["omega", "v", "tau", "tau_imp"]], w["modes"][["omega", "v", "tau", "tau_imp"]])
    assert r["geometry"]["faces"] == w["geometry"]["faces"]
    assert r["detectors"]["n"] == (2, 2, 2)
    a = oracle.trace(w, n=3000, threads=4)
    b = oracle.trace(r, n=3000, threads=4)
    assert np.array_equal(a["counts"], b["counts"])
    assert np.array_equal(a["raw"], b["raw"])


def test_mat_data_formats_and_the_impurity_column(tmp_path):
    f1 = tmp_path / "m1.txt"
    f1.write_text("# omega dos v domega tau pol tau_imp\n"
                  "1.0e12, 2.0e3, 8000, 1e11, 1e-10, 1, 5e-9\n"
                  "1.0e12 1.0e3 4000 1e11 2e-10 2 5e-9\n"
                  "2.0e12 4.0e3 7000 1e11 5e-11 1 1e-9\n")
    m = P.read_mat_data(str(f1), 1)
    assert list(m["bin"]) == [0, 0, 1] and list(m["branch"]) == [1, 2, 1]
    assert m["tau_imp"][2] == 1e-9 and m["dos"][1] == 1.0e3
    f2 = tmp_path / "m2.txt"
    f2.write_text("1e13 6400 1.5625e-11 1e6\n")
    m2 = P.read_mat_data(str(f2), 2)
    assert m2["C"][0] == 1e6 and m2["tau_imp"][0] == 0.0
    with pytest.raises(ValueError):
        P.read_mat_data(str(f2), 1)


def test_the_papers_nanomesh_files(tmp_path):
    """The example the paper's I/O section describes: a 34 x 34 x 22 nm cell, periodic in x and y,
    diffuse top and bottom, four internal line walls (an 11-nm square pore), N = 1e6,
    N_scat^max = 10, V = 2.28e-23 m^3, T_lin = 300 K."""
    (tmp_path / "Out_bnd.txt").write_text("34e-9 34e-9 22e-9\n")
    (tmp_path / "In_bnd.txt").write_text("11.5e-9 11.5e-9 22.5e-9 11.5e-9 0 -1 0\n"
                                         "22.5e-9 11.5e-9 22.5e-9 22.5e-9 1 0 0\n"
                                         "22.5e-9 22.5e-9 11.5e-9 22.5e-9 0 1 0\n"
                                         "11.5e-9 22.5e-9 11.5e-9 11.5e-9 -1 0 0\n")
    (tmp_path / "Boundary_prop.txt").write_text(
        "1 3 0 34e-9 0\n2 3 -34e-9 0 0\n3 3 0 -34e-9 0\n4 3 34e-9 0 0\n5 2 0 0 0\n6 2 0 0 0\n"
        "7 2 0 0 0\n8 2 0 0 0\n9 2 0 0 0\n10 2 0 0 0\n")
    (tmp_path / "Thermal_gradient.txt").write_text("1 3 0 -2.94e6 0\n")
    (tmp_path / "Sim_param.txt").write_text("1000000 10 2.28e-23 300\n")
    (tmp_path / "mat_data.txt").write_text("1e13 6400 1.5625e-11 1e6\n")
    w = P.read_case(str(tmp_path), fmt=2)
    assert [c[6] for c in w["geometry"]["walls"]] == [7, 8, 9, 10]
    assert w["geometry"]["walls"][1][:6] == (22.5e-9, 11.5e-9, 22.5e-9, 22.5e-9, 1.0, 0.0)
    r = oracle.trace(W.with_(w, **{"problem.N": 2000}), threads=4)
    c = dict(zip(oracle.COUNT_NAMES, r["counts"]))
    p_rej = (11e-9 / 34e-9) ** 2                 # the square pore's share of the cell
    assert abs(c["rejections"] / 2000 - p_rej / (1 - p_rej)) < 4 * (p_rej / (1 - p_rej) ** 2 / 2000) ** 0.5
    assert c["diffuse"] > 0
    # written back and read again: the same case
    P.write_case(w, str(tmp_path / "again"))
    w2 = P.read_case(str(tmp_path / "again"), fmt=2)
    assert w2["geometry"]["walls"] == [tuple(float(x) for x in c[:6]) + (c[6], 2, float(c[8]), 0.0)
                                       for c in w["geometry"]["walls"]]
    assert w["problem"]["N"] == 1000000 and w["problem"]["n_scat_max"] == 10
    assert w["geometry"]["volume"] == 2.28e-23 and w["problem"]["T_lin"] == 300.0
    assert w["geometry"]["gradT"] == (0.0, -2.94e6, 0.0) and w["problem"]["score_axis"] == 1
    assert not w["problem"]["transient"]
    oracle.Tables(w)       # a valid problem


def test_results_files(tmp_path):
    """Steady: one row per detector and one column per frequency bin (rows of a bin summed);
    detector_location lists the cuboids with the last axis fastest, as the tallies' cells."""
    w = _box_case()
    w["modes"] = W.silicon_like_modes(300.0, n_bins=10)
    w["problem"]["format"] = 1
    M = len(w["modes"])
    T = np.arange(8 * M, dtype=float).reshape(8, M)
    q = np.stack([T, 2 * T, 3 * T], -1)
    files = P.write_results(w, {"T": T, "q": q}, str(tmp_path))
    assert [os.path.basename(f) for f in files] == ["detector_location.txt", "T300.txt", "Qx300.txt",
                                                    "Qy300.txt", "Qz300.txt"]
    loc = np.loadtxt(files[0])
    assert loc.shape == (8, 6)
    assert np.allclose(loc[1], [0, 5e-8, 0, 5e-8, 5e-8, 1e-7]) and np.allclose(loc[2], [0, 5e-8, 5e-8, 1e-7, 0, 5e-8])
    Tb = np.loadtxt(files[1])
    assert Tb.shape == (8, 10)
    bins = w["modes"]["bin"]
    assert np.allclose(Tb[3, 2], T[3, bins == 2].sum())
    assert np.allclose(np.loadtxt(files[3]), 2 * Tb)
