"""Small analytic test scenes (data only) for the oracle pins and parity cases."""
import math

import numpy as np

import workloads as W


def plane_scene(material=W.MAT_MIRROR, ior=1.5, half=4.0, z=0.0, normal_up=True):
    """One flat square [-half, half]^2 at height z made of two triangles
    (object 0), vertex normals equal to the face normal."""
    v = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float64)
    if normal_up:
        t = np.array([[0, 1, 2], [0, 2, 3]])
        n = np.tile([0, 0, 1.0], (4, 1))
    else:
        t = np.array([[0, 2, 1], [0, 3, 2]])
        n = np.tile([0, 0, -1.0], (4, 1))
    return W._finish("plane", v, n, t, np.zeros(2), [material], [ior], np.zeros((0, 4)), [], 2 * half)


def strip_profile(x):
    """y-invariant wavy profile z = f(x) and its slope."""
    f = 0.15 * np.sin(2.3 * x) + 0.08 * np.sin(5.1 * x + 0.7)
    df = 0.15 * 2.3 * np.cos(2.3 * x) + 0.08 * 5.1 * np.cos(5.1 * x + 0.7)
    return f, df


def strip_scene(material=W.MAT_MIRROR, ior=1.5, nx=241, x0=-3.0, x1=3.0, y_half=3.0):
    """y-invariant wavy surface z = f(x) over [x0, x1] x [-y_half, y_half]:
    nx vertices in x, two rows in y (so every triangle spans the full y
    range), vertex normals from the exact slope.  Object 0."""
    xs = np.linspace(x0, x1, nx)
    f, df = strip_profile(xs)
    V, N = [], []
    for y in (-y_half, y_half):
        for x, z, d in zip(xs, f, df):
            V.append([x, y, z])
            n = np.array([-d, 0.0, 1.0])
            N.append(n / np.linalg.norm(n))
    T = []
    for i in range(nx - 1):
        a, b, c, d = i, i + 1, nx + i + 1, nx + i
        T += [[a, b, c], [a, c, d]]
    return W._finish("strip", np.array(V), np.array(N), np.array(T), np.zeros(len(T)), [material], [ior],
                     np.zeros((0, 4)), [], x1 - x0)


def endpoints(xD, xL, n=1, types=0, nD=(0, 0, 1), obj1=-1):
    xD = np.atleast_2d(np.asarray(xD, np.float64))
    xL = np.atleast_2d(np.asarray(xL, np.float64))
    N = max(len(xD), len(xL))
    xD = np.broadcast_to(xD, (N, 3))
    xL = np.broadcast_to(xL, (N, 3))
    nd = np.broadcast_to(np.asarray(nD, np.float64), (N, 3))
    return W._pack(xD, nd, xL, np.full(N, n), np.full(N, types), np.full(N, obj1))
