"""Reader of trained 3D Gaussian scenes stored as PLY files (the scenes of Sec. 4.1).

The de-facto layout of trained 3DGS scenes: one `vertex` element, one
property per scalar, binary little-endian (ASCII is accepted too):

    x y z                      centre
    f_dc_0 f_dc_1 f_dc_2       degree-0 SH coefficient of R, G, B
    f_rest_0 ... f_rest_{3(K-1)-1}
                               the other SH coefficients, channel-major:
                               f_rest[c * (K - 1) + (k - 1)] is coefficient k of channel c
    opacity                    logit of the peak opacity (sigma = sigmoid)
    scale_0 scale_1 scale_2    log of the scaling vector
    rot_0 rot_1 rot_2 rot_3    rotation quaternion (w, x, y, z), not normalised
    (nx ny nz and any other properties are ignored)

K = (degree + 1)^2 follows from the number of f_rest properties.  The SH
coefficients are those of the real basis with the Condon-Shortley sign (the
basis the library evaluates), so a trained scene renders with its own colours.

`read_ply` returns the library's layout (fp32, structure of arrays, the SH
coefficients as rows k * 3 + c); `write_ply` writes that layout back.  Host
IO only: no arithmetic of the render path happens here.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np

_TYPES = {"char": "i1", "int8": "i1", "uchar": "u1", "uint8": "u1", "short": "i2", "int16": "i2",
          "ushort": "u2", "uint16": "u2", "int": "i4", "int32": "i4", "uint": "u4", "uint32": "u4",
          "float": "f4", "float32": "f4", "double": "f8", "float64": "f8"}


@dataclasses.dataclass
class PlyGaussians:
    """Gaussian parameters in the library's layout (see GaussianTensors.from_scene)."""
    means: np.ndarray           # [3][n]
    log_scales: np.ndarray      # [3][n]
    quats: np.ndarray           # [4][n]  (w, x, y, z)
    opacity_logits: np.ndarray  # [n]
    sh: np.ndarray              # [3 K][n], row k * 3 + c
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])


def _parse_header(f):
    first = f.readline()
    if first.strip() != b"ply":
        raise ValueError("not a PLY file (no 'ply' magic line)")
    fmt = None
    elements = []  # [name, count, [(type, name)]]
    while True:
        line = f.readline()
        if not line:
            raise ValueError("PLY header has no end_header line")
        words = line.decode("ascii", errors="replace").split()
        if not words or words[0] in ("comment", "obj_info"):
            continue
        if words[0] == "end_header":
            break
        if words[0] == "format":
            fmt = words[1]
        elif words[0] == "element":
            elements.append([words[1], int(words[2]), []])
        elif words[0] == "property":
            if not elements:
                raise ValueError("PLY property before any element")
            if words[1] == "list":
                raise ValueError(f"list property '{words[-1]}' is not supported in element '{elements[-1][0]}'")
            if words[1] not in _TYPES:
                raise ValueError(f"unknown PLY property type '{words[1]}'")
            elements[-1][2].append((words[1], words[2]))
    if fmt not in ("binary_little_endian", "binary_big_endian", "ascii"):
        raise ValueError(f"unsupported PLY format '{fmt}'")
    return fmt, elements, f.tell()


def read_ply(path) -> PlyGaussians:
    with open(path, "rb") as f:
        fmt, elements, data_start = _parse_header(f)
    if not elements or elements[0][0] != "vertex":
        raise ValueError("the first PLY element must be 'vertex'")
    _, n, props = elements[0]
    endian = ">" if fmt == "binary_big_endian" else "<"
    dtype = np.dtype([(name, endian + _TYPES[t]) for t, name in props])
    if fmt == "ascii":
        table = np.loadtxt(path, skiprows=_header_lines(path), max_rows=n, ndmin=2)
        if table.shape[1] < len(props):
            raise ValueError("ASCII PLY rows hold fewer values than the header declares")
        data = np.zeros(n, dtype)
        for j, (_, name) in enumerate(props):
            data[name] = table[:, j]
    else:
        need = data_start + n * dtype.itemsize
        if os.path.getsize(path) < need:
            raise ValueError(f"PLY file is truncated: {os.path.getsize(path)} bytes, the vertices need {need}")
        data = np.memmap(path, dtype=dtype, mode="r", offset=data_start, shape=(n,))
    names = set(dtype.names)
    required = ["x", "y", "z", "opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3",
                "f_dc_0", "f_dc_1", "f_dc_2"]
    missing = [r for r in required if r not in names]
    if missing:
        raise ValueError(f"PLY vertex element lacks {missing}")
    rest = sorted((int(nm[len("f_rest_"):]) for nm in names if nm.startswith("f_rest_")))
    if rest != list(range(len(rest))):
        raise ValueError("f_rest_* properties are not numbered 0 .. m-1")
    if len(rest) % 3:
        raise ValueError(f"{len(rest)} f_rest properties: not a multiple of 3")
    per_channel = len(rest) // 3
    degree = {0: 0, 3: 1, 8: 2, 15: 3}.get(per_channel)
    if degree is None:
        raise ValueError(f"{per_channel} f_rest coefficients per channel: no SH degree up to 3 has that many")
    K = (degree + 1) ** 2
    col = lambda nm: np.asarray(data[nm], np.float32)  # noqa: E731
    means = np.stack([col("x"), col("y"), col("z")])
    log_scales = np.stack([col(f"scale_{i}") for i in range(3)])
    quats = np.stack([col(f"rot_{i}") for i in range(4)])
    logits = col("opacity").copy()
    sh = np.empty((3 * K, n), np.float32)
    for c in range(3):
        sh[c] = col(f"f_dc_{c}")
        for k in range(1, K):
            sh[k * 3 + c] = col(f"f_rest_{c * (K - 1) + (k - 1)}")
    return PlyGaussians(np.ascontiguousarray(means), np.ascontiguousarray(log_scales), np.ascontiguousarray(quats),
                        logits, sh, degree)


def _header_lines(path) -> int:
    count = 0
    with open(path, "rb") as f:
        for line in f:
            count += 1
            if line.strip() == b"end_header":
                return count
    raise ValueError("PLY header has no end_header line")


def write_ply(path, g, binary=True):
    """Writes Gaussians in the library's layout (anything with means, log_scales, quats, opacity_logits, sh and
    sh_degree as numpy arrays) as a PLY file of the layout above, normals zero."""
    means = np.asarray(g.means, np.float32)
    n = means.shape[1]
    K = (int(g.sh_degree) + 1) ** 2
    sh = np.asarray(g.sh, np.float32).reshape(3 * K, n)
    names = ["x", "y", "z", "nx", "ny", "nz", "f_dc_0", "f_dc_1", "f_dc_2"]
    names += [f"f_rest_{i}" for i in range(3 * (K - 1))]
    names += ["opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3"]
    data = np.zeros(n, np.dtype([(nm, "<f4") for nm in names]))
    for i, nm in enumerate("xyz"):
        data[nm] = means[i]
    for c in range(3):
        data[f"f_dc_{c}"] = sh[c]
        for k in range(1, K):
            data[f"f_rest_{c * (K - 1) + (k - 1)}"] = sh[k * 3 + c]
    data["opacity"] = np.asarray(g.opacity_logits, np.float32)
    for i in range(3):
        data[f"scale_{i}"] = np.asarray(g.log_scales, np.float32)[i]
    for i in range(4):
        data[f"rot_{i}"] = np.asarray(g.quats, np.float32)[i]
    fmt = "binary_little_endian" if binary else "ascii"
    header = "ply\nformat " + fmt + " 1.0\nelement vertex " + str(n) + "\n"
    header += "".join(f"property float {nm}\n" for nm in names) + "end_header\n"
    with open(path, "wb") as f:
        f.write(header.encode("ascii"))
        if binary:
            f.write(data.tobytes())
        else:
            np.savetxt(f, np.stack([data[nm] for nm in names], axis=1), fmt="%.9g")
