"""FP64 oracle for the discretised acoustic FWI / LSRTM problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states the continuous problem (Section "FWI and LSRTM"): the
constant-density acoustic equation m u_tt - Lap u = s with zero initial
data and non-reflecting boundaries (eq. FWD), m = 1/c^2, the data
f(m) = R F(m) and misfit J = 1/2 ||f - g||^2 (eq. FWI), the Born
linearisation with source -m_r u0_tt (eq. Born, eq. LSRTM), the adjoint
equation driven by -R^*(f - g) (eq. FWI_adj) and the gradient
dJ/dm = -int u_tt v dt (eq. adj_grad1).

Here the problem is discretised and then differentiated exactly
("discretise, then optimise"):

* padded grid: ``nb`` sponge cells on all four sides; the model is
  extended by edge replication (m_pad = P m) and the reported gradient is
  P^T applied to the padded one;
* Laplacian: centred 8th-order second difference on each axis, the field
  is zero outside the padded grid;
* sponge: sigma = sigma_max (xi_x^2 + xi_z^2) with xi the depth into the
  layer in cells divided by nb, sigma_max = 3 vref ln(1/R) / (2 nb h);
  st = sigma dt / 2, A = 1/(1+st), B = (1-st)/(1+st), K = A dt^2 / m_pad;
* leapfrog: u^{n+1} = 2A u^n - B u^{n-1} + K (Lap u^n + s^n), u^0 = u^-1 = 0,
  i.e. (m/dt^2)[(1+st)u^{n+1} - 2u^n + (1-st)u^{n-1}] - Lap u^n = s^n;
* point source s^n = w[n] / h^2 at one node; data d[n] = u^{n+1} at the
  receiver nodes (time (n+1) dt);
* exact discrete adjoint: lam^n = 2A lam^{n+1} - B lam^{n+2}
  + K (Lap lam^{n+1} - R^T r^n), lam^nt = lam^{nt+1} = 0, r = d - d_obs;
* gradient: g_pad = sum_n lam^n * q^n with q^n = (Lap u^n + s^n)/m_pad
  (q is u_tt by the equation, lam is -v of eq. FWI_adj up to scaling);
* stable domain: the leapfrog scheme is stable only for velocities up to the
  bound that comes with the geometry (vmax_bound, the CFL condition), so the
  scheme sees m_eff = max(m, 1/vmax_bound^2) everywhere (the misfit is then
  finite for every positive model), and the gradient is that of
  J(m_eff(m)): the folded gradient times the mask [m >= 1/vmax_bound^2]
  (the derivative from above at the floor, where projected iterates sit);
  Born modelling linearises the same map (dm masked the same way).  For
  models inside the bound nothing changes.
"""
from __future__ import annotations

import numpy as np

# Centred 8th-order weights for the second derivative: c0, then c1..c4 for
# the symmetric pairs at distance 1..4.
C8 = np.array([-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0])


# ----------------------------------------------------------------------------
# grid, sponge and model extension
# ----------------------------------------------------------------------------

def sponge_xi(n_interior: int, nb: int) -> np.ndarray:
    """Depth into the sponge, in cells, divided by nb, for each padded index."""
    i = np.arange(n_interior + 2 * nb)
    depth = np.zeros(i.shape, dtype=np.float64)
    left = i < nb
    right = i >= nb + n_interior
    depth[left] = nb - i[left]
    depth[right] = i[right] - (nb + n_interior - 1)
    return depth / nb


def sponge(geom):
    """Damping coefficients A, B on the padded grid (FP64)."""
    if geom.refl >= 1.0:
        smax = 0.0
    else:
        smax = 3.0 * geom.vref * np.log(1.0 / geom.refl) / (2.0 * geom.nb * geom.h)
    xz = sponge_xi(geom.nz, geom.nb)[:, None]
    xx = sponge_xi(geom.nx, geom.nb)[None, :]
    st = smax * (xz ** 2 + xx ** 2) * geom.dt / 2.0
    return 1.0 / (1.0 + st), (1.0 - st) / (1.0 + st)


def model_floor(geom) -> float:
    """Smallest m for which the scheme is stable: 1 / vmax_bound^2."""
    return 1.0 / float(geom.vmax_bound) ** 2


def effective_model(geom, m):
    """(m_eff, mask): the model the scheme uses, max(m, floor), and the
    derivative of that map, 1 where m >= floor (from above at the floor
    itself, where projected iterates sit) and 0 below it."""
    m = np.asarray(m, np.float64)
    f = model_floor(geom)
    return np.maximum(m, f), (m >= f).astype(np.float64)


def pad_model(m: np.ndarray, nb: int) -> np.ndarray:
    """P m: replicate the edge values into the sponge (corners take corners)."""
    return np.pad(np.asarray(m, np.float64), nb, mode="edge")


def fold(g_pad: np.ndarray, nz: int, nx: int, nb: int) -> np.ndarray:
    """P^T g: add every padded cell onto the interior cell it was copied from."""
    iz = np.clip(np.arange(nz + 2 * nb) - nb, 0, nz - 1)
    ix = np.clip(np.arange(nx + 2 * nb) - nb, 0, nx - 1)
    out = np.zeros((nz, nx))
    np.add.at(out, (iz[:, None], ix[None, :]), g_pad)
    return out


# ----------------------------------------------------------------------------
# Laplacian
# ----------------------------------------------------------------------------

def _shift(u, k, axis, periodic):
    """v[i] = u[i + k] along ``axis``; zero outside unless periodic."""
    if periodic:
        return np.roll(u, -k, axis=axis)
    v = np.zeros_like(u)
    n = u.shape[axis]
    src = [slice(None)] * u.ndim
    dst = [slice(None)] * u.ndim
    if k > 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    v[tuple(dst)] = u[tuple(src)]
    return v


def laplacian(u: np.ndarray, h: float, periodic: bool = False) -> np.ndarray:
    out = 2.0 * C8[0] * u
    for j in range(1, 5):
        for axis in (0, 1):
            out = out + C8[j] * (_shift(u, j, axis, periodic) + _shift(u, -j, axis, periodic))
    return out / (h * h)


# ----------------------------------------------------------------------------
# propagation
# ----------------------------------------------------------------------------

def _pads(geom, m):
    m_pad = pad_model(effective_model(geom, m)[0], geom.nb)
    A, B = sponge(geom)
    K = A * geom.dt ** 2 / m_pad
    return m_pad, A, B, K


def _src_node(geom, s):
    return int(geom.src_iz[s]) + geom.nb, int(geom.src_ix[s]) + geom.nb


def _rec_nodes(geom, s):
    return (np.asarray(geom.rec_iz[s], np.int64) + geom.nb,
            np.asarray(geom.rec_ix[s], np.int64) + geom.nb)


def forward_shot(geom, m, s, keep_q=False, periodic=False, u_init=None, src_on=True):
    """One shot of the forward scheme.

    Returns (d [nt, R], q list or None, final (u^nt, u^{nt-1})).  ``u_init``
    optionally gives (u^0, u^-1) for the energy and dispersion checks.
    """
    m_pad, A, B, K = _pads(geom, m)
    shape = m_pad.shape
    if u_init is None:
        u, u_prev = np.zeros(shape), np.zeros(shape)
    else:
        u, u_prev = (np.array(a, np.float64) for a in u_init)
    sz, sx = _src_node(geom, s)
    rz, rx = _rec_nodes(geom, s)
    w = np.asarray(geom.wavelet, np.float64)
    d = np.zeros((geom.nt, rz.shape[0]))
    qs = [] if keep_q else None
    for n in range(geom.nt):
        rhs = laplacian(u, geom.h, periodic)
        if src_on:
            rhs[sz, sx] += w[n] / geom.h ** 2
        if keep_q:
            qs.append(rhs / m_pad)
        u_next = 2.0 * A * u - B * u_prev + K * rhs
        d[n] = u_next[rz, rx]
        u_prev, u = u, u_next
    return d, qs, (u, u_prev)


def forward_model(geom, m):
    """f(m) = R F(m) for every shot: d [S, nt, R]."""
    return np.stack([forward_shot(geom, m, s)[0] for s in range(geom.nshots)])


def misfit(d, d_obs):
    r = np.asarray(d, np.float64) - np.asarray(d_obs, np.float64)
    return 0.5 * float(np.sum(r * r))


def adjoint_shot(geom, m, s, r, qs):
    """Run the exact discrete adjoint for one shot and image against q.

    r [nt, R] is the adjoint source (the data residual), qs the list of
    q^n = (Lap u^n + s^n)/m_pad from the forward run.  Returns the padded,
    unfolded gradient sum_n lam^n * q^n.
    """
    m_pad, A, B, K = _pads(geom, m)
    rz, rx = _rec_nodes(geom, s)
    lam1 = np.zeros(m_pad.shape)  # lam^{n+1}
    lam2 = np.zeros(m_pad.shape)  # lam^{n+2}
    g = np.zeros(m_pad.shape)
    r = np.asarray(r, np.float64)
    for n in range(geom.nt - 1, -1, -1):
        inj = np.zeros(m_pad.shape)
        np.add.at(inj, (rz, rx), r[n])
        lam = 2.0 * A * lam1 - B * lam2 + K * (laplacian(lam1, geom.h) - inj)
        g += lam * qs[n]
        lam2, lam1 = lam1, lam
    return g


def adjoint_gradient(geom, m, d_obs):
    """(J, dJ/dm) with dJ/dm on the interior grid (after P^T)."""
    J = 0.0
    g_pad = np.zeros((geom.nz_p, geom.nx_p))
    for s in range(geom.nshots):
        d, qs, _ = forward_shot(geom, m, s, keep_q=True)
        r = d - np.asarray(d_obs[s], np.float64)
        J += 0.5 * float(np.sum(r * r))
        g_pad += adjoint_shot(geom, m, s, r, qs)
    return J, fold(g_pad, geom.nz, geom.nx, geom.nb) * effective_model(geom, m)[1]


def adjoint_from_residual(geom, m, r):
    """Gradient of <r, f(m)> with respect to m, i.e. J'(m)^T r (FP64)."""
    g_pad = np.zeros((geom.nz_p, geom.nx_p))
    for s in range(geom.nshots):
        _, qs, _ = forward_shot(geom, m, s, keep_q=True)
        g_pad += adjoint_shot(geom, m, s, r[s], qs)
    return fold(g_pad, geom.nz, geom.nx, geom.nb) * effective_model(geom, m)[1]


# ----------------------------------------------------------------------------
# Born modelling and its adjoint (eq. Born, eq. LSRTM)
# ----------------------------------------------------------------------------

def born_shot(geom, m0, dm, s):
    """Scattered data L dm for one shot: du solves the forward scheme with the
    source -(P dm) * q0^n, where q0^n = (Lap u0^n + s^n)/m0_pad."""
    m_pad, A, B, K = _pads(geom, m0)
    dm_pad = pad_model(np.asarray(dm, np.float64) * effective_model(geom, m0)[1], geom.nb)
    sz, sx = _src_node(geom, s)
    rz, rx = _rec_nodes(geom, s)
    w = np.asarray(geom.wavelet, np.float64)
    u, u_prev = np.zeros(m_pad.shape), np.zeros(m_pad.shape)
    du, du_prev = np.zeros(m_pad.shape), np.zeros(m_pad.shape)
    d = np.zeros((geom.nt, rz.shape[0]))
    for n in range(geom.nt):
        rhs = laplacian(u, geom.h)
        rhs[sz, sx] += w[n] / geom.h ** 2
        q0 = rhs / m_pad
        du_next = 2.0 * A * du - B * du_prev + K * (laplacian(du, geom.h) - dm_pad * q0)
        u_next = 2.0 * A * u - B * u_prev + K * rhs
        d[n] = du_next[rz, rx]
        u_prev, u = u, u_next
        du_prev, du = du, du_next
    return d


def born(geom, m0, dm):
    return np.stack([born_shot(geom, m0, dm, s) for s in range(geom.nshots)])


def born_adjoint(geom, m0, y):
    """L^T y = P^T sum_s sum_n lam^n * q0^n with lam driven by y (at m0)."""
    return adjoint_from_residual(geom, m0, y)


# ----------------------------------------------------------------------------
# general linear source -> data map and its adjoint (for the dot-product test)
# ----------------------------------------------------------------------------

def rtm_filter(image, h):
    """Laplacian-filtered RTM image (Section "Numerical Example", the LSRTM
    comparison): -Lap_h of the image with the 8th-order second differences,
    zero outside the interior grid."""
    return -laplacian(np.asarray(image, np.float64), h)


def scaled_rtm_start(geom, m0, d_r):
    """The filtered RTM image f = rtm_filter(L^T d_r) scaled by the alpha that
    minimises ||alpha L f - d_r||: a starting model for LSRTM."""
    f = rtm_filter(born_adjoint(geom, m0, d_r), geom.h)
    lf = born(geom, m0, f)
    alpha = float(np.sum(lf * d_r) / np.sum(lf * lf))
    return alpha * f, alpha


def source_to_data(geom, m, src_field, s=0):
    """d = R u for an arbitrary space-time source field src_field [nt, nz_p, nx_p]
    entering as K * src^n (no point source)."""
    m_pad, A, B, K = _pads(geom, m)
    rz, rx = _rec_nodes(geom, s)
    u, u_prev = np.zeros(m_pad.shape), np.zeros(m_pad.shape)
    d = np.zeros((geom.nt, rz.shape[0]))
    for n in range(geom.nt):
        u_next = 2.0 * A * u - B * u_prev + K * (laplacian(u, geom.h) + src_field[n])
        d[n] = u_next[rz, rx]
        u_prev, u = u, u_next
    return d


def data_to_source(geom, m, y, s=0):
    """Adjoint of :func:`source_to_data`: returns -lam^n for n = 0..nt-1."""
    m_pad, A, B, K = _pads(geom, m)
    rz, rx = _rec_nodes(geom, s)
    lam1, lam2 = np.zeros(m_pad.shape), np.zeros(m_pad.shape)
    out = np.zeros((geom.nt,) + m_pad.shape)
    for n in range(geom.nt - 1, -1, -1):
        inj = np.zeros(m_pad.shape)
        np.add.at(inj, (rz, rx), y[n])
        lam = 2.0 * A * lam1 - B * lam2 + K * (laplacian(lam1, geom.h) - inj)
        out[n] = -lam
        lam2, lam1 = lam1, lam
    return out


# ----------------------------------------------------------------------------
# closed forms used as pins
# ----------------------------------------------------------------------------

def energy(u_next, u, m_pad, h, dt):
    """Discrete energy at n+1/2 of the undamped, source-free scheme:
    1/2 ||(u^{n+1}-u^n)/dt||_m^2 + 1/2 <u^{n+1}, -Lap u^n>."""
    du = (u_next - u) / dt
    return 0.5 * float(np.sum(m_pad * du * du)) - 0.5 * float(np.sum(u_next * laplacian(u, h)))


def green_2d_trace(t, r, v, wavelet_fn):
    """Homogeneous 2D Green's function convolved with w, at distance r:
    u(r,t) = (1/2pi) int_0^{acosh(v t / r)} w(t - (r/v) cosh th) d th, t > r/v."""
    from scipy.integrate import quad
    out = np.zeros(len(t))
    for i, ti in enumerate(t):
        if v * ti <= r:
            continue
        top = np.arccosh(v * ti / r)
        val, _ = quad(lambda th: wavelet_fn(ti - (r / v) * np.cosh(th)), 0.0, top, limit=400)
        out[i] = val / (2.0 * np.pi)
    return out
