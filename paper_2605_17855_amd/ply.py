"""Trained-scene ingestion: the binary PLY files that 3D Gaussian Splatting training writes.

The paper renders trained Gaussian models (its table of evaluated scenes).  Those files hold
one vertex per Gaussian with float properties

    x y z                     centre
    nx ny nz                  unused (zeros)
    f_dc_0 f_dc_1 f_dc_2      degree-0 SH coefficient per colour channel
    f_rest_0 ...              the higher-degree coefficients, channel-major:
                              f_rest_{c (B - 1) + (k - 1)} is basis k >= 1 of channel c,
                              B = (deg + 1)^2
    opacity                   logit of the opacity
    scale_0 scale_1 scale_2   log standard deviation per axis
    rot_0 rot_1 rot_2 rot_3   rotation quaternion (w, x, y, z), not normalised

and evaluate colour as sum_k coef_k Y_k(dir) + 0.5 with the real spherical harmonics in the
Condon-Shortley phase, which is the basis (index l*l + l + m) and offset the renderer uses,
so the coefficients carry over unchanged.  `load_ply` maps a file onto a `scenes.Scene`
(opacity through the logistic function, quaternion normalised); `save_ply` writes the
inverse.  Only the binary little-endian encoding is read.
"""
from __future__ import annotations

import math
import os

import numpy as np

from .scenes import Scene

_PLY_TYPES = {"float": "<f4", "float32": "<f4", "double": "<f8", "float64": "<f8", "uchar": "u1", "uint8": "u1",
              "char": "i1", "int8": "i1", "ushort": "<u2", "uint16": "<u2", "short": "<i2", "int16": "<i2",
              "uint": "<u4", "uint32": "<u4", "int": "<i4", "int32": "<i4"}


def _read_header(f):
    lines = []
    while True:
        line = f.readline()
        if not line:
            raise ValueError("PLY header has no end_header")
        line = line.decode("ascii", errors="replace").strip()
        lines.append(line)
        if line == "end_header":
            return lines, f.tell()


def load_ply(path: str) -> Scene:
    """The Gaussians of a trained-scene PLY file as a Scene (float32 arrays)."""
    with open(path, "rb") as f:
        if f.readline().strip() != b"ply":
            raise ValueError(f"{path}: not a PLY file")
        lines, offset = _read_header(f)
    fmt = next((ln.split()[1] for ln in lines if ln.startswith("format ")), None)
    if fmt != "binary_little_endian":
        raise ValueError(f"{path}: PLY format {fmt!r} (binary_little_endian expected)")
    n, fields, in_vertex, before = None, [], False, 0
    for ln in lines:
        parts = ln.split()
        if parts[0] == "element":
            in_vertex = parts[1] == "vertex"
            if in_vertex:
                n = int(parts[2])
            elif n is None:
                raise ValueError(f"{path}: element {parts[1]!r} before the vertices is not supported")
        elif parts[0] == "property" and in_vertex:
            if parts[1] == "list":
                raise ValueError(f"{path}: list property in the vertex element")
            if parts[1] not in _PLY_TYPES:
                raise ValueError(f"{path}: property type {parts[1]!r}")
            fields.append((parts[2], _PLY_TYPES[parts[1]]))
    if n is None:
        raise ValueError(f"{path}: no vertex element")
    dtype = np.dtype(fields)
    v = np.memmap(path, dtype=dtype, mode="r", offset=offset, shape=(n,)) if n else np.zeros(0, dtype)
    names = set(dtype.names or ())

    def col(name):
        if name not in names:
            raise ValueError(f"{path}: vertex property {name!r} missing")
        return np.asarray(v[name], np.float64)

    rest = sorted((int(nm[len("f_rest_"):]) for nm in names if nm.startswith("f_rest_")))
    if rest != list(range(len(rest))) or len(rest) % 3:
        raise ValueError(f"{path}: f_rest properties are not 3 (B - 1) consecutive indices")
    nb = len(rest) // 3 + 1
    deg = int(round(math.sqrt(nb))) - 1
    if (deg + 1) ** 2 != nb or deg > 3:
        raise ValueError(f"{path}: {len(rest)} f_rest coefficients do not give SH degree 0..3")
    mean = np.stack([col("x"), col("y"), col("z")])
    log_scale = np.stack([col(f"scale_{i}") for i in range(3)])
    quat = np.stack([col(f"rot_{i}") for i in range(4)])
    norm = np.linalg.norm(quat, axis=0, keepdims=True)
    quat = np.where(norm > 0, quat / np.where(norm > 0, norm, 1.0), np.array([[1.0], [0.0], [0.0], [0.0]]))
    opacity = 1.0 / (1.0 + np.exp(-col("opacity")))
    sh = np.zeros((nb, 3, n), np.float64)
    for c in range(3):
        sh[0, c] = col(f"f_dc_{c}")
        for k in range(1, nb):
            sh[k, c] = col(f"f_rest_{c * (nb - 1) + (k - 1)}")
    return Scene(mean.astype(np.float32), log_scale.astype(np.float32), quat.astype(np.float32),
                 opacity.astype(np.float32), sh.astype(np.float32), deg)


def save_ply(scene: Scene, path: str) -> None:
    """Writes the scene in the trained-scene PLY layout (binary little endian)."""
    n, nb = scene.n, (scene.sh_degree + 1) ** 2
    names = (["x", "y", "z", "nx", "ny", "nz"] + [f"f_dc_{c}" for c in range(3)]
             + [f"f_rest_{i}" for i in range(3 * (nb - 1))] + ["opacity"] + [f"scale_{i}" for i in range(3)]
             + [f"rot_{i}" for i in range(4)])
    rec = np.zeros(n, np.dtype([(nm, "<f4") for nm in names]))
    for i, nm in enumerate("xyz"):
        rec[nm] = scene.mean[i]
    sh = np.asarray(scene.sh, np.float32).reshape(nb, 3, n)
    for c in range(3):
        rec[f"f_dc_{c}"] = sh[0, c]
        for k in range(1, nb):
            rec[f"f_rest_{c * (nb - 1) + (k - 1)}"] = sh[k, c]
    o = np.clip(np.asarray(scene.opacity, np.float64), 1e-12, 1.0 - 1e-12)
    rec["opacity"] = np.log(o / (1.0 - o))
    for i in range(3):
        rec[f"scale_{i}"] = scene.log_scale[i]
    for i in range(4):
        rec[f"rot_{i}"] = scene.quat[i]
    header = "ply\nformat binary_little_endian 1.0\nelement vertex %d\n" % n
    header += "".join(f"property float {nm}\n" for nm in names) + "end_header\n"
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        f.write(header.encode("ascii"))
        f.write(rec.tobytes())
    os.replace(tmp, path)
