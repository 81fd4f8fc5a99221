"""Independent brute-force single step of the lattice-BGK update (numpy).

Used only to pin the C oracle.  Written separately from it and in a different
style:
  * push streaming: every departing population is moved along its velocity
    and, if its path ends inside the wall or body, reflected by tracing
    where the bounced particle lands (the C oracle pulls instead);
  * the collision builds the Hermite basis H0, H1, H2 explicitly and
    projects the non-equilibrium part onto H2 with einsum (Sec. 5, eqs.
    feq_h2, fne, regularization).
Geometry conventions: half-way walls; plate wall at y = -1/2 moving with
U_w along x, x periodic, a stationary wall at y = ny - 1/2 or an open
rest-equilibrium far field; box = solid cells [x0,x0+lx) x [y0,y0+ly).
"""
import numpy as np


def _reflect_box(p, d, box):
    """Arrival cell of a population leaving fluid cell p whose straight
    destination d is solid.  Per axis: a departure coordinate outside the
    body's range is mirrored through the face plane, else kept."""
    x0, y0, lx, ly = box
    lo = (x0, y0)
    hi = (x0 + lx, y0 + ly)
    a = []
    for k in range(2):
        if p[k] < lo[k]:
            a.append(2 * lo[k] - 1 - d[k])
        elif p[k] >= hi[k]:
            a.append(2 * hi[k] - 1 - d[k])
        else:
            a.append(p[k])
    return tuple(a)


def _box_side(p, box):
    """Face a population leaving fluid cell p towards the body hits: 'b',
    't' (below, above: p within the body's x range), 'l', 'r' (left, right:
    within its y range), or None (outside both ranges: a corner)."""
    x0, y0, lx, ly = box
    inx = x0 <= p[0] < x0 + lx
    iny = y0 <= p[1] < y0 + ly
    if inx and not iny:
        return "b" if p[1] < y0 else "t"
    if iny and not inx:
        return "l" if p[0] < x0 else "r"
    return None


def stream(f, v, w, theta, geometry, far, box, U, rho0, diffuse=False, sigma=1.0):
    """Push streaming.  Returns (f_adv, Fx, Fy); f is [q][y][x].  With
    diffuse=True the plate wall, or each face of the box, re-emits what hits
    it as the H2 equilibrium at the wall velocity, at the density that returns
    the column's mass; with sigma < 1 only that fraction is re-emitted
    diffusely and the rest of each particle is reflected specularly (the
    normal velocity reversed); the box's corners keep bounce-back."""
    Q, ny, nx = f.shape
    opp = [int(np.flatnonzero((v[:, 0] == -v[i, 0]) & (v[:, 1] == -v[i, 1]))[0]) for i in range(Q)]
    refl = [int(np.flatnonzero((v[:, 0] == v[i, 0]) & (v[:, 1] == -v[i, 1]))[0]) for i in range(Q)]
    wall_in = np.zeros_like(f)  # arrivals from the diffuse / specular wall
    fadv = np.full_like(f, np.nan)
    Fx = Fy = 0.0

    def solid(x, y):
        if geometry != "box":
            return False
        x0, y0, lx, ly = box
        return x0 <= x < x0 + lx and y0 <= y < y0 + ly

    # diffuse plate wall: mass hitting the wall per column, and emitted shape
    hit = np.zeros(nx)
    box_hits = []  # (q, departure, destination, bounce-back arrival, value, bounce-back out)
    if diffuse and geometry == "plate":
        for q in range(Q):
            for y in range(ny):
                if y + v[q, 1] < 0:
                    hit += f[q, y, :]
        vu = v[:, 0] * U
        eq = 1 + vu / theta + vu ** 2 / (2 * theta ** 2) - U ** 2 / (2 * theta)
        per_rho = sum(v[i, 1] * w[i] * eq[i] for i in range(Q) if v[i, 1] > 0)
        rho_w = hit / per_rho
    for q in range(Q):
        ux, uy = int(v[q, 0]), int(v[q, 1])
        for y in range(ny):
            for x in range(nx):
                if solid(x, y):
                    continue
                val = f[q, y, x]
                dx, dy = x + ux, y + uy
                if geometry == "plate":
                    dx %= nx
                    if dy < 0:
                        # bounces on the moving wall; arrives with velocity -u
                        i = opp[q]
                        ax, ay = x, -1 - dy
                        if diffuse:
                            # incoming momentum now; the arrivals' outgoing
                            # momentum once they are all in place
                            wall_in[i, ay, ax] += sigma * w[i] * rho_w[x] * eq[i]
                            j = refl[q]
                            wall_in[j, ay, (x + ux) % nx] += (1 - sigma) * val
                            Fx += ux * val
                            Fy += uy * val
                            continue
                        out = val + 2 * w[i] * rho0 * (v[i, 0] * U) / theta
                        fadv[i, ay, ax] = out
                        Fx += -v[i, 0] * (val + out)
                        Fy += -v[i, 1] * (val + out)
                        continue
                    if dy >= ny:
                        if far == "wall":
                            fadv[opp[q], 2 * ny - 1 - dy, x] = val
                        continue
                    fadv[q, dy, dx] = val
                elif geometry == "periodic":
                    fadv[q, dy % ny, dx % nx] = val
                else:
                    if not (0 <= dx < nx and 0 <= dy < ny):
                        continue
                    if solid(dx, dy):
                        i = opp[q]
                        ax, ay = _reflect_box((x, y), (dx, dy), box)
                        out = val + 2 * w[i] * rho0 * (v[i, 0] * U) / theta
                        if diffuse and _box_side((x, y), box) is not None:
                            box_hits.append((q, x, y, dx, dy, ax, ay, val, out))
                            continue
                        fadv[i, ay, ax] = out
                        Fx += -v[i, 0] * (val + out)
                        Fy += -v[i, 1] * (val + out)
                        continue
                    fadv[q, dy, dx] = val
    if diffuse and geometry == "box":
        # box faces: a population that hits a face (its departure beside the
        # body on one axis only) is gathered per face column -- the column
        # of the cell bounce-back would send it to -- with the mass
        # bounce-back would deliver; the diffuse share of each column goes
        # out as the H2 equilibrium at the wall velocity in the bounce-back
        # directions, the specular share goes to the destination mirrored
        # through the face plane with the normal velocity reversed (plus the
        # moving-wall term on the faces normal to the motion)
        vu = v[:, 0] * U
        eq = 1 + vu / theta + vu ** 2 / (2 * theta ** 2) - U ** 2 / (2 * theta)
        refx = [int(np.flatnonzero((v[:, 0] == -v[i, 0]) & (v[:, 1] == v[i, 1]))[0])
                for i in range(Q)]
        mass, shape = {}, {}
        for q, x, y, dx, dy, ax, ay, val, out in box_hits:
            key = (_box_side((x, y), box), ax if _box_side((x, y), box) in "bt" else ay)
            mass[key] = mass.get(key, 0.0) + out
            shape[key] = shape.get(key, 0.0) + w[opp[q]] * eq[opp[q]]
        arrivals = np.zeros_like(f)
        for q, x, y, dx, dy, ax, ay, val, out in box_hits:
            side = _box_side((x, y), box)
            key = (side, ax if side in "bt" else ay)
            i = opp[q]
            arrivals[i, ay, ax] += sigma * w[i] * mass[key] / shape[key] * eq[i]
            x0, y0, lx, ly = box
            if side in "bt":
                plane = y0 if side == "b" else y0 + ly
                j, mx, my = refl[q], dx, 2 * plane - 1 - dy
                extra = 0.0
            else:
                plane = x0 if side == "l" else x0 + lx
                j, mx, my = refx[q], 2 * plane - 1 - dx, dy
                extra = 2 * w[j] * rho0 * (v[j, 0] * U) / theta
            arrivals[j, my, mx] += (1 - sigma) * (val + extra)
            Fx += v[q, 0] * val
            Fy += v[q, 1] * val
        for q, x, y, dx, dy, ax, ay, val, out in box_hits:
            i = opp[q]
            fadv[i, ay, ax] = arrivals[i, ay, ax]
            Fx -= v[i, 0] * arrivals[i, ay, ax]
            Fy -= v[i, 1] * arrivals[i, ay, ax]
    if diffuse and geometry == "plate":
        for i in range(Q):
            for y in range(ny):
                if y < v[i, 1]:  # arrival rows of the wall
                    fadv[i, y, :] = wall_in[i, y, :]
                    Fx -= v[i, 0] * wall_in[i, y, :].sum()
                    Fy -= v[i, 1] * wall_in[i, y, :].sum()
    # whatever was not delivered comes from the rest-equilibrium far field
    hole = np.isnan(fadv)
    fadv[hole] = (w[:, None, None] * rho0 * np.ones_like(f))[hole]
    if geometry == "box":
        x0, y0, lx, ly = box
        fadv[:, y0:y0 + ly, x0:x0 + lx] = 0.0
    return fadv, Fx, Fy


def collide(fadv, v, w, theta, tau, regularized=True):
    """Collision on a [q][y][x] field with the explicit Hermite basis."""
    vv = v.astype(np.float64)
    H1 = vv                                             # [Q,2]
    H2 = vv[:, :, None] * vv[:, None, :] - theta * np.eye(2)[None]  # [Q,2,2]
    rho = fadv.sum(0)
    j = np.einsum("qyx,qa->ayx", fadv, vv)
    with np.errstate(invalid="ignore", divide="ignore"):
        u = np.where(rho != 0, j / np.where(rho != 0, rho, 1), 0.0)
    # equilibrium, eq. feq_h2, written as a Hermite expansion
    a1 = rho * u                                        # [2,y,x]
    a2 = rho[None, None] * u[:, None] * u[None, :]      # [2,2,y,x]
    feq = w[:, None, None] * (rho[None]
                              + np.einsum("qa,ayx->qyx", H1, a1) / theta
                              + np.einsum("qab,abyx->qyx", H2, a2) / (2 * theta ** 2))
    keep = 1.0 - (0.0 if np.isinf(tau) else 1.0 / tau)
    if not regularized:
        return feq + keep * (fadv - feq)
    A = np.einsum("qyx,qa,qb->abyx", fadv - feq, vv, vv)
    fne = w[:, None, None] * np.einsum("qab,abyx->qyx", H2, A) / (2 * theta ** 2)
    return feq + keep * fne


def step(f, v, w, theta, tau, geometry, far, box, U, rho0=1.0, regularized=True, diffuse=False,
         sigma=1.0):
    fadv, Fx, Fy = stream(f, v, w, theta, geometry, far, box, U, rho0, diffuse, sigma)
    out = collide(fadv, v, w, theta, tau, regularized)
    if geometry == "box":
        x0, y0, lx, ly = box
        out[:, y0:y0 + ly, x0:x0 + lx] = 0.0
    return out, Fx, Fy
