"""Exact rational 2DSW step on tiny grids (test infrastructure only; ``fractions.Fraction``).

A second, independent statement of the same step as the C oracle, written in
face-flux (scatter) form: every active face moves a volume of water from one cell
to its neighbour, and the Shapiro filter is an exchange across each active face.
The C oracle gathers per cell instead. With exact arithmetic, any index, sign or
upwinding slip in either form shows up as a disagreement.

Step (a reading of Sect. 6.2, which names the predictor "dyn", the first-order
Shapiro filter and the velocity update but prints no equations):
  1. each active face gets its predicted velocity from the pressure gradient;
  2. the face carries velocity x upwind total depth (old surface) for one time step,
     taken from the upstream cell and given to the downstream cell;
  3. each active face exchanges eps/4 of the surface difference of its two cells;
  4. the new velocities are the predicted ones; land and inactive faces hold zero.
"""

from __future__ import annotations

from fractions import Fraction


def _fr(x) -> Fraction:
    return Fraction(float(x))


def step(nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v):
    """One exact step. Array arguments are nested lists (or arrays) indexed [j][i];
    returns (eta, u, v) as nested lists of Fractions."""
    dx, dy, g, dt, eps = _fr(dx), _fr(dy), _fr(g), _fr(dt), _fr(eps)
    wet = [[bool(mask[j][i]) for i in range(nx)] for j in range(ny)]
    Hq = [[_fr(H[j][i]) for i in range(nx)] for j in range(ny)]
    e0 = [[_fr(eta[j][i]) for i in range(nx)] for j in range(ny)]
    u0 = [[_fr(u[j][i]) for i in range(nx)] for j in range(ny)]
    v0 = [[_fr(v[j][i]) for i in range(nx)] for j in range(ny)]
    zero = Fraction(0)

    u1 = [[zero] * nx for _ in range(ny)]
    v1 = [[zero] * nx for _ in range(ny)]
    es = [[e0[j][i] if wet[j][i] else zero for i in range(nx)] for j in range(ny)]

    # faces between (j,i) and (j,i+1): x-direction; between (j,i) and (j+1,i): y-direction
    faces = []
    for j in range(ny):
        for i in range(nx - 1):
            if wet[j][i] and wet[j][i + 1]:
                faces.append(((j, i), (j, i + 1), u0[j][i], dx, u1))
    for j in range(ny - 1):
        for i in range(nx):
            if wet[j][i] and wet[j + 1][i]:
                faces.append(((j, i), (j + 1, i), v0[j][i], dy, v1))

    for (a, b, vel, d, out) in faces:
        (ja, ia), (jb, ib) = a, b
        vs = vel - g * dt * (e0[jb][ib] - e0[ja][ia]) / d
        out[ja][ia] = vs
        if vs > 0:
            depth = Hq[ja][ia] + e0[ja][ia]
        else:
            depth = Hq[jb][ib] + e0[jb][ib]
        moved = dt * vs * depth / d  # surface change carried across the face in one step
        es[ja][ia] -= moved
        es[jb][ib] += moved

    e1 = [row[:] for row in es]
    quarter = eps / 4
    for (a, b, _vel, _d, _out) in faces:
        (ja, ia), (jb, ib) = a, b
        x = quarter * (es[jb][ib] - es[ja][ia])
        e1[ja][ia] += x
        e1[jb][ib] -= x
    for j in range(ny):
        for i in range(nx):
            if not wet[j][i]:
                e1[j][i] = zero
    return e1, u1, v1


def run(nx, ny, dx, dy, g, dt, eps, H, mask, eta, u, v, nsteps):
    e, uu, vv = eta, u, v
    for _ in range(nsteps):
        e, uu, vv = step(nx, ny, dx, dy, g, dt, eps, H, mask, e, uu, vv)
    return e, uu, vv
