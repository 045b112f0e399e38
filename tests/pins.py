"""Independent checkers that pin the oracle (test infrastructure).

Each routine here is written from textbook mathematics, not from the
oracle's code: the forward lens map (Sec. 2.1 lens equation), the
Paczynski point-lens magnification, the Witt & Mao (1994) uniform-disk
point-lens magnification, a radial quadrature of the same quantity from
first principles, critical curves and caustics from |f'(z)| = 1, and
brute-force inverse ray shooting of the image area.
"""
import numpy as np
from scipy import integrate, special


def lens_setup(s, q):
    m1 = 1.0 / (1.0 + q)
    m2 = q / (1.0 + q)
    z1 = -q * s / (1.0 + q)
    z2 = s / (1.0 + q)
    return m1, m2, z1, z2


def forward_map(s, q, z):
    """Source position of image position z (CM frame), Sec. 2.1 lens equation."""
    m1, m2, z1, z2 = lens_setup(s, q)
    z = np.asarray(z, dtype=np.complex128)
    return z + m1 / (np.conj(z1) - np.conj(z)) + m2 / (np.conj(z2) - np.conj(z))


def jacobian(s, q, z):
    m1, m2, z1, z2 = lens_setup(s, q)
    fp = m1 / (z1 - z) ** 2 + m2 / (z2 - z) ** 2
    return 1.0 - np.abs(fp) ** 2


def paczynski(u):
    u = np.asarray(u, dtype=np.float64)
    return (u * u + 2.0) / (u * np.sqrt(u * u + 4.0))


def witt_mao(u, rho):
    """Uniform disk of radius rho at distance u from a unit point lens."""
    if abs(u - rho) < 1e-14:
        return 2.0 / (np.pi * rho) + (1 + rho * rho) / (np.pi * rho * rho) * (
            np.pi / 2 + np.arcsin((rho * rho - 1) / (rho * rho + 1)))
    if u == 0.0:
        return np.sqrt(1 + 4 / rho ** 2)
    n = 4 * u * rho / (u + rho) ** 2
    S = np.sqrt(4 + (u - rho) ** 2)
    m = 4 * n / (4 + (u - rho) ** 2)
    K = special.ellipk(m)
    E = special.ellipe(m)
    Pi = special.elliprf(0.0, 1 - m, 1.0) + n / 3.0 * special.elliprj(0.0, 1 - m, 1.0, 1 - n)
    return (1 / np.pi) * ((u + rho) * S / (2 * rho ** 2) * E
                          - (u - rho) * (8 + u * u - rho * rho) / (2 * rho * rho * S) * K
                          + 2 * (u - rho) ** 2 * (1 + rho * rho) / (rho * rho * (u + rho) * S) * Pi)


def disk_point_lens_radial(u, rho, weight=None):
    """(1/pi rho^2) * integral over the disk of mu(w) [weight(r)], by polar
    coordinates about the lens: w is the distance from the lens, the arc of
    the circle of radius w inside the disk has angle L(w)."""
    def arc(w):
        if u == 0.0:
            return 2 * np.pi if w <= rho else 0.0
        c = (w * w + u * u - rho * rho) / (2 * w * u)
        if c <= -1:
            return 2 * np.pi
        if c >= 1:
            return 0.0
        return 2 * np.arccos(c)

    def integrand(w):
        return w * paczynski(w) * arc(w)

    pts = sorted({abs(u - rho), u + rho})
    lo = 0.0
    total = 0.0
    for hi in pts:
        if hi > lo:
            v, _ = integrate.quad(integrand, lo, hi, epsabs=0, epsrel=1e-13, limit=500)
            total += v
        lo = hi
    return total / (np.pi * rho * rho)


def critical_curve(s, q, nphi=4096):
    """Points z with |f'(z)| = 1: roots of m1(z-z2)^2 + m2(z-z1)^2 =
    e^{i phi} (z-z1)^2 (z-z2)^2 for phi on a grid."""
    m1, m2, z1, z2 = lens_setup(s, q)
    out = []
    for phi in np.linspace(0, 2 * np.pi, nphi, endpoint=False):
        e = np.exp(1j * phi)
        # e (z-z1)^2 (z-z2)^2 - m1 (z-z2)^2 - m2 (z-z1)^2 = 0
        p12 = np.polymul([1, -z1], [1, -z1])
        p22 = np.polymul([1, -z2], [1, -z2])
        quart = e * np.polymul(p12, p22)
        quart = np.polyadd(quart, -m1 * p22)
        quart = np.polyadd(quart, -m2 * p12)
        out.append(np.roots(quart))
    return np.concatenate(out)


def caustic(s, q, nphi=4096):
    z = critical_curve(s, q, nphi)
    return forward_map(s, q, z)


def ray_shoot_area(s, q, zc, rho, box, n0=512, depth=7, sub=4):
    """Area of the image-plane region mapping inside the disk |zeta - zc| <=
    rho, by inverse ray shooting on an adaptive quadtree.  A cell is taken
    whole (inside or outside) only when the source-plane distance of its
    centre from the limb exceeds twice a Lipschitz bound of the lens map
    over the cell, (h/sqrt 2)(1 + |f'|); otherwise it is split.  At the last
    level a sub x sub grid of rays gives the covered fraction."""
    m1, m2, z1, z2 = lens_setup(s, q)
    x0, x1, y0, y1 = box
    h = (x1 - x0) / n0
    ny = int(np.ceil((y1 - y0) / h))
    cx = x0 + (np.arange(n0) + 0.5) * h
    cy = y0 + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(cx, cy, indexing="ij")
    cells = (X.ravel() + 1j * Y.ravel())
    area = 0.0

    def dist(z):
        with np.errstate(all="ignore"):
            return np.abs(forward_map(s, q, z) - zc) - rho

    for level in range(depth + 1):
        with np.errstate(all="ignore"):
            fp = np.abs(m1 / (z1 - cells) ** 2 + m2 / (z2 - cells) ** 2)
        lip = 2.0 * (h / np.sqrt(2.0)) * (1.0 + fp)
        d = dist(cells)
        whole_in = np.isfinite(d) & (d < -lip)
        whole_out = np.isfinite(d) & (d > lip)
        area += whole_in.sum() * h * h
        mixed = cells[~whole_in & ~whole_out]
        if level == depth:
            g = (np.arange(sub) + 0.5) / sub - 0.5
            gx, gy = np.meshgrid(g, g, indexing="ij")
            frac = np.zeros(mixed.size)
            for o in (gx.ravel() + 1j * gy.ravel()) * h:
                frac += dist(mixed + o) <= 0
            area += frac.sum() / (sub * sub) * h * h
            break
        h /= 2
        q4 = np.array([1 + 1j, 1 - 1j, -1 + 1j, -1 - 1j]) * (h / 2)
        cells = (mixed[None, :] + q4[:, None]).ravel()
    return area


def real_images_newton(s, q, zeta, tol=1e-12):
    """All solutions of the lens equation zeta = z + conj(f(z)) by Newton's
    method on the real 2-D system from many starting points; independent of
    any polynomial.  The Newton step solves dz + conj(f') conj(dz) = -F."""
    m1, m2, z1, z2 = lens_setup(s, q)
    g = np.linspace(-3, 3, 61)
    X, Y = np.meshgrid(g, g)
    starts = [(X + 1j * Y).ravel()]
    for zl in (z1, z2):
        for r in np.geomspace(1e-5, 1.0, 30):
            starts.append(zl + r * np.exp(1j * np.linspace(0, 2 * np.pi, 24, endpoint=False)))
    z = np.concatenate(starts)
    with np.errstate(all="ignore"):
        for _ in range(200):
            F = forward_map(s, q, z) - zeta
            fp = m1 / (z1 - z) ** 2 + m2 / (z2 - z) ** 2
            J = 1 - np.abs(fp) ** 2
            dz = -(F - np.conj(fp) * np.conj(F)) / J
            step = np.abs(dz)
            cap = np.minimum(0.1, 0.5 * np.minimum(np.abs(z - z1), np.abs(z - z2)))
            dz = np.where(step > cap, dz * cap / step, dz)
            z = z + dz
        F = np.abs(forward_map(s, q, z) - zeta)
        fp = np.abs(m1 / (z1 - z) ** 2 + m2 / (z2 - z) ** 2)
    # rounding of z is amplified by |f'| near a lens
    ok = np.isfinite(F) & (F < tol * (1 + np.abs(zeta) + fp * np.abs(z)))
    sols = []
    for zz in z[ok]:
        if all(abs(zz - t) > 1e-7 for t in sols):
            sols.append(zz)
    return np.array(sols)
