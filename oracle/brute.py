"""Pure-Python loop versions of the forward model for tiny inputs (TEST INFRASTRUCTURE ONLY).

Written separately from the vectorised oracle (no shared helpers) so that the two pin each other:
explicit edge comparisons instead of floor, linear scans over nodes instead of searchsorted, a
stable insertion sort instead of argsort, and literal per-particle / per-bin / per-corner loops.
Same readings as the vectorised oracle (Sec. 3 pipeline; see rubix_oracle's module docstring).
"""
from __future__ import annotations

import math

C_KMS = 299792.458


def rotation(phi1, phi2, phi3):
    """Rz(phi3) Ry(phi2) Rx(phi1) by explicit 3x3 matrix products (nested lists)."""
    def mm(a, b):
        return [[sum(a[i][k] * b[k][j] for k in range(3)) for j in range(3)] for i in range(3)]
    c1, s1 = math.cos(phi1), math.sin(phi1)
    c2, s2 = math.cos(phi2), math.sin(phi2)
    c3, s3 = math.cos(phi3), math.sin(phi3)
    rx = [[1, 0, 0], [0, c1, -s1], [0, s1, c1]]
    ry = [[c2, 0, s2], [0, 1, 0], [-s2, 0, c2]]
    rz = [[c3, -s3, 0], [s3, c3, 0], [0, 0, 1]]
    return mm(rz, mm(ry, rx))


def spaxel_index(xp, yp, nx, ny, s):
    """Cell by explicit comparisons against the cell edges of the centred grid (half-open)."""
    tx = xp / s + nx / 2.0
    ty = yp / s + ny / 2.0
    ix = iy = None
    for k in range(nx):
        if k <= tx < k + 1:
            ix = k
    for k in range(ny):
        if k <= ty < k + 1:
            iy = k
    if ix is None or iy is None:
        return nx * ny
    return iy * nx + ix


def stable_sort(keys):
    """Insertion sort of indices by key (stable by construction)."""
    order = []
    for i, k in enumerate(keys):
        pos = len(order)
        while pos > 0 and keys[order[pos - 1]] > k:
            pos -= 1
        order.insert(pos, i)
    return order


def _bracket(u, nodes):
    """Clamp u, then find the node interval by a linear scan; right-hand cell at interior nodes."""
    n = len(nodes)
    if u <= nodes[0]:
        return 0, 0.0
    if u >= nodes[-1]:
        return n - 2, 1.0
    for j in range(n - 1):
        if nodes[j] <= u < nodes[j + 1]:
            return j, (u - nodes[j]) / (nodes[j + 1] - nodes[j])
    raise AssertionError("unreachable")


def particle_flux(age, met, mass, vlos, log_age_nodes, met_nodes, flux, ssp_start, ssp_step,
                  lam_tel, z_sys=0.0, flux_scale=1.0):
    """Observed spectrum of one particle at each telescope wavelength, literal loops."""
    ja, ta = _bracket(math.log10(age), log_age_nodes)
    jz, tz = _bracket(met, met_nodes)
    n = len(flux[0][0])
    beta = vlos / C_KMS
    jac = 1.0 / ((1.0 + z_sys) * (1.0 + beta))
    out = []
    for lam in lam_tel:
        lam_rest = lam / ((1.0 + z_sys) * (1.0 + beta))
        # locate the SSP node interval containing lam_rest by scanning node wavelengths
        val = 0.0
        for k in range(n - 1):
            lo = ssp_start + k * ssp_step
            hi = ssp_start + (k + 1) * ssp_step
            last = (k == n - 2)
            if lo <= lam_rest < hi or (last and lam_rest == hi):
                tau = (lam_rest - lo) / ssp_step
                for da, wa in ((0, 1.0 - ta), (1, ta)):
                    for dz, wz in ((0, 1.0 - tz), (1, tz)):
                        row = flux[ja + da][jz + dz]
                        val += wa * wz * ((1.0 - tau) * row[k] + tau * row[k + 1])
                break
        out.append(flux_scale * mass * jac * val)
    return out


def cube(parts, angles, nx, ny, s, lam_tel, log_age_nodes, met_nodes, flux, ssp_start,
         ssp_step):
    """Raw cube [ny*nx][n_tel] as nested lists: per particle, per bin, per corner."""
    R = rotation(*angles)
    c = [[0.0] * len(lam_tel) for _ in range(nx * ny)]
    for (x, y, z, vx, vy, vz, m, age, met) in parts:
        xp = R[0][0] * x + R[0][1] * y + R[0][2] * z
        yp = R[1][0] * x + R[1][1] * y + R[1][2] * z
        key = spaxel_index(xp, yp, nx, ny, s)
        if key == nx * ny:
            continue
        vlos = R[2][0] * vx + R[2][1] * vy + R[2][2] * vz
        f = particle_flux(age, met, m, vlos, log_age_nodes, met_nodes, flux, ssp_start,
                          ssp_step, lam_tel)
        for j, v in enumerate(f):
            c[key][j] += v
    return c


def gauss_conv_1d(seq, sigma):
    """Zero-padded sampled-Gaussian smoothing of a list, radius int(4 sigma + 0.5)."""
    if sigma <= 0:
        return list(seq)
    r = int(4.0 * sigma + 0.5)
    w = [math.exp(-0.5 * (k / sigma) ** 2) for k in range(-r, r + 1)]
    tot = sum(w)
    w = [x / tot for x in w]
    n = len(seq)
    out = []
    for i in range(n):
        acc = 0.0
        for k in range(-r, r + 1):
            if 0 <= i + k < n:
                acc += w[k + r] * seq[i + k]
        out.append(acc)
    return out
