"""Exact laws of tiny MPR systems, by quadrature, for pinning the sampler.

TEST INFRASTRUCTURE (part of the CPU oracle; only tests may import it).

The Gibbs density of the MPR model is proportional to exp(-H/T) with H of
Eq. (3) (Secs. 2.1-2.2).  On a 3 x 3 grid the checkerboard colours make the
sites of one colour conditionally independent given the other colour, so
the marginals reduce to low-dimensional integrals that Gauss-Legendre
quadrature evaluates to near machine precision.  In 1D with q = 1 the open
chain's bond angles are independent von Mises variables and the specific
energy is -I_1(beta)/I_0(beta) (Sec. 5.1.2, Eq. 16); for q = 1/2 the open
chain is integrated with a transfer matrix.

Grid convention: site (y, x); 3 x 3 corners (0,0), (0,2), (2,0), (2,2);
edges (0,1), (1,0), (1,2), (2,1); centre (1,1).
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _nodes(nbins, per_bin):
    """Gauss-Legendre nodes and weights on [0, 2*pi], ``per_bin`` per bin."""
    x, w = np.polynomial.legendre.leggauss(per_bin)
    edges = np.linspace(0.0, TWO_PI, nbins + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    nodes = (0.5 * (hi - lo) * x[None, :] + 0.5 * (hi + lo)).ravel()
    weights = (0.5 * (hi - lo) * w[None, :]).ravel()
    return nodes, weights


def _bond(beta, q, a, b):
    """exp(beta (cos(q (a - b)) - 1)): one bond's Boltzmann factor, scaled by
    exp(-beta) so that products of many bonds stay finite."""
    return np.exp(beta * (np.cos(q * (a - b)) - 1.0))


def _bin_probs(density, weights, nbins):
    mass = (density * weights).reshape(nbins, -1).sum(axis=1)
    return mass / mass.sum()


def single_site_bins(nbr_angles, beta, q, nbins=8, per_bin=48):
    """Bin probabilities of one free site whose neighbours are frozen at
    ``nbr_angles``: density proportional to prod_j exp(beta cos q(phi - phi_j))."""
    x, w = _nodes(nbins, per_bin)
    dens = np.ones_like(x)
    for a in nbr_angles:
        dens = dens * _bond(beta, q, x, a)
    return _bin_probs(dens, w, nbins)


def single_site_moments(nbr_angles, beta, q, n=256):
    """Mean and variance of the angle of one free site whose neighbours are
    frozen at ``nbr_angles``, under the density proportional to
    prod_j exp(beta cos q(phi - phi_j)) on [0, 2*pi): Gauss-Legendre
    quadrature with ``n`` nodes per eighth of the circle."""
    x, w = _nodes(8, n)
    dens = np.ones_like(x)
    for a in nbr_angles:
        dens = dens * _bond(beta, q, x, a)
    m0 = float((dens * w).sum())
    m1 = float((dens * w * x).sum()) / m0
    m2 = float((dens * w * x * x).sum()) / m0
    return m1, m2 - m1 * m1


EDGE_CORNERS = {(0, 1): ((0, 0), (0, 2)), (1, 0): ((0, 0), (2, 0)),
                (1, 2): ((0, 2), (2, 2)), (2, 1): ((2, 0), (2, 2))}


def corners_frozen_bins(corners, beta, q, nbins=8, per_bin=40):
    """3 x 3 grid with the four corners frozen at ``corners[(y, x)]``; the
    centre and the four edges are free.  Returns (centre bins, dict of edge
    bins)."""
    x, w = _nodes(nbins, per_bin)
    # g[e][c_idx] = integral over the edge angle given the centre angle
    wedge = {}
    g = {}
    for e, (k1, k2) in EDGE_CORNERS.items():
        fe = _bond(beta, q, x, corners[k1]) * _bond(beta, q, x, corners[k2])      # (E,)
        wedge[e] = fe
        joint = _bond(beta, q, x[:, None], x[None, :]) * fe[:, None]            # (E, C)
        g[e] = (joint * w[:, None]).sum(axis=0)                                  # (C,)
    centre = np.prod([g[e] for e in g], axis=0)
    out_c = _bin_probs(centre, w, nbins)
    out_e = {}
    for e in g:
        others = np.prod([g[f] for f in g if f != e], axis=0)                   # (C,)
        joint = _bond(beta, q, x[:, None], x[None, :]) * wedge[e][:, None] * others[None, :]
        out_e[e] = _bin_probs((joint * w[None, :]).sum(axis=1), w, nbins)
    return out_c, out_e


def free3x3(beta, q, nbins=8, per_bin=16):
    """Fully free 3 x 3 grid (unconditional).  Returns (centre bins, log Z)
    where Z is the scaled partition function (each bond carries
    exp(-beta)), so that <H> = -d log Z / d beta - 12.

    Given the centre angle c, the edges and corners form a ring
    corner - edge - corner - ... ; integrating each edge out gives the kernel
    G_c(k, k') = sum_e w_e b(e, c) b(e, k) b(e, k'), and the ring integral
    over the corners is trace((G_c W)^4).
    """
    x, w = _nodes(nbins, per_bin)
    B = _bond(beta, q, x[:, None], x[None, :])          # (E, K): b(e, k)
    dens = np.empty_like(x)
    for i, c in enumerate(x):
        a = _bond(beta, q, x, c) * w                     # (E,)
        G = (B * a[:, None]).T @ B                        # (K, K)
        M = G * w[None, :]
        M2 = M @ M
        dens[i] = np.trace(M2 @ M2)
    logZ = math.log(float((dens * w).sum()))
    return _bin_probs(dens, w, nbins), logZ


def free3x3_specific_energy(beta, q, h=1e-5, **kw):
    """Exact e = <H>/N_GP of the fully free 3 x 3 grid (N_GP = 12), by a
    central difference of log Z in beta."""
    lp = free3x3(beta + h, q, **kw)[1]
    lm = free3x3(beta - h, q, **kw)[1]
    return (-(lp - lm) / (2 * h) - 12.0) / 12.0


def chain1d_energy_q1(beta):
    """Eq. (16): e = -I_1(beta)/I_0(beta) for the open q = 1 chain."""
    from scipy.special import ive
    return -ive(1, beta) / ive(0, beta)


def chain1d_specific_energy(beta, q, n, nbins=16, per_bin=24, h=1e-5):
    """Exact e = <H>/(n - 1) of an open chain of n free sites, any q, by a
    transfer matrix on Gauss-Legendre nodes and a central difference."""
    x, w = _nodes(nbins, per_bin)

    def log_z(b):
        K = _bond(b, q, x[:, None], x[None, :]) * w[None, :]
        v = w.copy()
        logs = 0.0
        for _ in range(n - 1):
            v = v @ K
            s = v.sum()
            logs += math.log(s)
            v = v / s
        return logs

    dlog = (log_z(beta + h) - log_z(beta - h)) / (2 * h)
    return (-dlog - (n - 1)) / (n - 1)


def uniform_gap_gap_cos(q):
    """E[cos q(phi_i - phi_j)] for two independent U[0, 2*pi) angles:
    |E e^{i q phi}|^2 = (sin(pi q) / (pi q))^2."""
    return (math.sin(math.pi * q) / (math.pi * q)) ** 2


def uniform_gap_sample_cos(q, phi_j):
    """E[cos q(phi - phi_j)] for phi ~ U[0, 2*pi) and a fixed phi_j:
    (sin(q (2*pi - phi_j)) + sin(q phi_j)) / (2*pi*q)."""
    return (math.sin(q * (TWO_PI - phi_j)) + math.sin(q * phi_j)) / (TWO_PI * q)


def gmrf_single_site_bins(nbr_angles, beta, nbins=8):
    """Bin probabilities of one free site of the GMRF variant (Sec. 4.4)
    whose n neighbours are frozen at ``nbr_angles``: the density
    prod_j exp(-beta (phi - phi_j)^2 / (2 pi^2)) on [0, 2 pi) is a normal
    density with mean m = mean(phi_j) and variance pi^2 / (beta n),
    truncated to [0, 2 pi); its bin masses follow from the error function.
    beta = 0 gives the uniform law."""
    edges = np.linspace(0.0, TWO_PI, nbins + 1)
    if beta == 0.0:
        return np.diff(edges) / TWO_PI
    m = float(np.mean(nbr_angles))
    sd = math.pi / math.sqrt(beta * len(nbr_angles))
    cdf = np.array([0.5 * math.erfc(-(e - m) / (sd * math.sqrt(2.0))) for e in edges])
    mass = np.diff(cdf)
    return mass / mass.sum()
