"""Plain FP64 oracle of the near-field layers and their Gaussian RBF interpolation.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

Section 3.3 replaces near-singular quadrature by interpolation: around each
vesicle of N points it places five layers of N target points, the membrane
points shifted along the normal by d in (-h, -h/2, 0, h/2, h), h the arclength
spacing; the single-layer velocity of that vesicle is known on the layers (the
paper predicts it with networks; here it is an input); and a Gaussian radial
basis function interpolant of those 5N values gives the velocity at any point of
the vesicle's near zone (Algorithm 4, interpolateInNearField).  The interpolant
is  s(x) = sum_a phi(|x - x_a|) c_a  with  phi(r) = exp(-r^2 / (eps h)^2)  and
coefficients from the symmetric positive definite system  K c = u,
K_ab = phi(|x_a - x_b|), solved by Cholesky factorisation.

Readings where the paper is silent (listed with the design notes):
  * h_v = sum_{j in v} w_j / N_v, the mean arclength spacing (as for the
    near-field rule of Section 2.2);
  * the normal is the outward unit normal, positive d outside the vesicle,
    whatever the orientation of the points (fixed by the sign of the enclosed
    signed area); the tangent comes from the spectral derivative of Section 2.2.1;
  * the Gaussian width is eps * h_v with eps a parameter (the paper gives none);
  * the 5N nodes of vesicle v sit at 5 * offsets[v] + l * N_v + k for layer l
    (d = (l - 2) h / 2) and membrane point k, in planar [2][5P] arrays;
  * a target near several vesicles receives the sum of their interpolants.
"""
import numpy as np
from scipy.linalg import solve_triangular

from oracle.spectral import spectral_derivative

LAYER_OFFSETS = (-1.0, -0.5, 0.0, 0.5, 1.0)  # in units of h


def vesicle_layers(x, w):
    """Five layers of one vesicle: x (2, N), w (N,) -> nodes (2, 5N), h."""
    n = x.shape[1]
    h = w.sum() / n
    xa = spectral_derivative(x)
    J = np.sqrt(xa[0] ** 2 + xa[1] ** 2)
    t = xa / J
    # enclosed signed area by the trapezoid rule of (x y_alpha - y x_alpha) / 2
    area = 0.5 * np.sum(x[0] * xa[1] - x[1] * xa[0]) * (2.0 * np.pi / n)
    s = 1.0 if area >= 0.0 else -1.0
    normal = s * np.stack([t[1], -t[0]])  # tangent turned clockwise: outward for a counter-clockwise curve
    nodes = np.concatenate([x + d * h * normal for d in LAYER_OFFSETS], axis=1)
    return nodes, h


def near_layers(X, w, offsets):
    """All vesicles: X (2, P), w (P,) -> layers (2, 5P), h (M,)."""
    X = np.asarray(X, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    P = X.shape[1]
    M = len(offsets) - 1
    layers = np.empty((2, 5 * P))
    h = np.zeros(M)
    for v in range(M):
        a, b = int(offsets[v]), int(offsets[v + 1])
        if b > a:
            layers[:, 5 * a:5 * b], h[v] = vesicle_layers(X[:, a:b], w[a:b])
    return layers, h


def gaussian(r2, width):
    """phi as a function of the squared distance."""
    return np.exp(-r2 / (width * width))


def kernel_matrix(nodes, width):
    d = nodes[:, :, None] - nodes[:, None, :]
    return gaussian(d[0] ** 2 + d[1] ** 2, width)


def vesicle_fit(nodes, values, width):
    """Coefficients c with K c = values (values (2, 5N)) by Cholesky, K = L L^T."""
    K = kernel_matrix(nodes, width)
    L = np.linalg.cholesky(K)
    y = solve_triangular(L, values.T, lower=True)
    return solve_triangular(L.T, y, lower=False).T


def rbf_fit(layers, layer_velocity, w, offsets, eps):
    """Coefficients of every vesicle, (2, 5P); the width of vesicle v is eps * h_v."""
    coeffs = np.zeros_like(np.asarray(layer_velocity, dtype=np.float64))
    for v in range(len(offsets) - 1):
        a, b = int(offsets[v]), int(offsets[v + 1])
        if b > a:
            h = np.sum(w[a:b]) / (b - a)
            sl = slice(5 * a, 5 * b)
            coeffs[:, sl] = vesicle_fit(layers[:, sl], layer_velocity[:, sl], eps * h)
    return coeffs


def vesicle_eval(nodes, coeffs, points, width):
    """s(points) for one vesicle's interpolant: points (2, Q) -> (2, Q)."""
    d = points[:, :, None] - nodes[:, None, :]
    G = gaussian(d[0] ** 2 + d[1] ** 2, width)
    return coeffs @ G.T


def rbf_eval_near(layers, coeffs, w, offsets, eps, targets, pairs):
    """u_near: for every near pair (target i, vesicle v) add v's interpolant at targets[:, i].

    pairs is an int array (K, 2).  Returns (2, P_targets)."""
    targets = np.asarray(targets, dtype=np.float64)
    out = np.zeros_like(targets)
    for i, v in np.asarray(pairs, dtype=np.int64).reshape(-1, 2):
        a, b = int(offsets[v]), int(offsets[v + 1])
        h = np.sum(w[a:b]) / (b - a)
        sl = slice(5 * a, 5 * b)
        out[:, i] += vesicle_eval(layers[:, sl], coeffs[:, sl], targets[:, i:i + 1], eps * h)[:, 0]
    return out
