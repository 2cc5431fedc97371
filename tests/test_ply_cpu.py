"""Trained-scene PLY ingestion (CPU): the attribute mapping of the trained-3DGS layout onto the
scene arrays, pinned by hand-built files with known values, and write/read round trips."""
import math

import numpy as np
import pytest

from paper_2605_17855_amd import ply, scenes


def _write(path, names, rows):
    header = "ply\nformat binary_little_endian 1.0\nelement vertex %d\n" % len(rows)
    header += "".join(f"property float {nm}\n" for nm in names) + "end_header\n"
    with open(path, "wb") as f:
        f.write(header.encode())
        f.write(np.asarray(rows, "<f4").tobytes())


def _names(deg):
    nb = (deg + 1) ** 2
    return (["x", "y", "z", "nx", "ny", "nz", "f_dc_0", "f_dc_1", "f_dc_2"]
            + [f"f_rest_{i}" for i in range(3 * (nb - 1))] + ["opacity", "scale_0", "scale_1", "scale_2"]
            + ["rot_0", "rot_1", "rot_2", "rot_3"])


def test_hand_built_file_maps_attributes(tmp_path):
    names = _names(3)
    idx = {nm: i for i, nm in enumerate(names)}
    row = np.zeros(len(names))
    row[idx["x"]], row[idx["y"]], row[idx["z"]] = 1.0, -2.0, 3.5
    row[idx["f_dc_0"]], row[idx["f_dc_1"]], row[idx["f_dc_2"]] = 0.25, -0.5, 0.75
    # channel-major higher coefficients: f_rest_{c*15 + k-1} is basis k of channel c
    row[idx["f_rest_0"]] = 1.0       # channel 0, basis 1
    row[idx["f_rest_15"]] = 2.0      # channel 1, basis 1
    row[idx["f_rest_44"]] = 3.0      # channel 2, basis 15
    row[idx["opacity"]] = 0.0        # logit 0 -> 0.5
    row[idx["scale_0"]], row[idx["scale_1"]], row[idx["scale_2"]] = math.log(0.1), 0.0, -1.0
    row[idx["rot_0"]], row[idx["rot_3"]] = 2.0, 2.0   # (w, x, y, z) = (2, 0, 0, 2) -> normalised
    row2 = np.zeros(len(names))
    row2[idx["opacity"]] = math.log(3.0)             # logit of 0.75
    row2[idx["rot_0"]] = 1.0
    _write(tmp_path / "a.ply", names, [row, row2])
    sc = ply.load_ply(str(tmp_path / "a.ply"))
    assert sc.n == 2 and sc.sh_degree == 3 and sc.sh.shape == (16, 3, 2)
    assert np.allclose(sc.mean[:, 0], [1.0, -2.0, 3.5])
    assert np.allclose(sc.sh[0, :, 0], [0.25, -0.5, 0.75])
    assert sc.sh[1, 0, 0] == 1.0 and sc.sh[1, 1, 0] == 2.0 and sc.sh[15, 2, 0] == 3.0
    assert np.count_nonzero(sc.sh[1:, :, 0]) == 3
    assert sc.opacity[0] == pytest.approx(0.5) and sc.opacity[1] == pytest.approx(0.75, rel=1e-6)
    assert np.allclose(sc.log_scale[:, 0], [math.log(0.1), 0.0, -1.0])
    assert np.allclose(sc.quat[:, 0], [math.sqrt(0.5), 0.0, 0.0, math.sqrt(0.5)])


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_degree_from_coefficient_count(tmp_path, deg):
    names = _names(deg)
    row = np.zeros(len(names))
    row[names.index("rot_0")] = 1.0
    _write(tmp_path / "d.ply", names, [row])
    assert ply.load_ply(str(tmp_path / "d.ply")).sh_degree == deg


def test_bad_files_raise(tmp_path):
    names = _names(1)[:-1]        # a missing rot_3
    _write(tmp_path / "m.ply", names, [np.zeros(len(names))])
    with pytest.raises(ValueError, match="rot_3"):
        ply.load_ply(str(tmp_path / "m.ply"))
    names = _names(0) + ["f_rest_0", "f_rest_1"]   # not a multiple of 3
    _write(tmp_path / "r.ply", names, [np.zeros(len(names))])
    with pytest.raises(ValueError, match="f_rest"):
        ply.load_ply(str(tmp_path / "r.ply"))
    (tmp_path / "t.ply").write_bytes(b"ply\nformat ascii 1.0\nelement vertex 0\nend_header\n")
    with pytest.raises(ValueError, match="binary_little_endian"):
        ply.load_ply(str(tmp_path / "t.ply"))


def test_round_trip(tmp_path):
    sc = scenes.clustered_scene(5000, seed=7, clusters=8)
    ply.save_ply(sc, str(tmp_path / "s.ply"))
    back = ply.load_ply(str(tmp_path / "s.ply"))
    assert back.n == sc.n and back.sh_degree == sc.sh_degree
    assert np.array_equal(back.mean, sc.mean) and np.array_equal(back.log_scale, sc.log_scale)
    assert np.array_equal(back.sh, sc.sh)
    assert np.allclose(back.quat, sc.quat, atol=1e-6)
    assert np.allclose(back.opacity, sc.opacity, rtol=1e-5, atol=1e-7)
    empty = scenes.clustered_scene(5000, seed=7, clusters=8).subset(np.zeros(0, np.int64))
    ply.save_ply(empty, str(tmp_path / "e.ply"))
    assert ply.load_ply(str(tmp_path / "e.ply")).n == 0
