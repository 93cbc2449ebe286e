"""Outer-loop optimiser: positivity transform and Adam (FP64 oracle).

App. B ("Iterative Optimiser"): Adam with default settings apart from the
learning rate (Kingma & Ba 2015: beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
bias-corrected moments) maximises the marginal likelihood; every
hyperparameter is reparameterised as theta = softplus(nu) = log(1 + exp(nu))
and the optimiser acts on nu.  The small workload's description instead
says "log-hyperparameters", so theta = exp(nu) is supported as well.
"""
from __future__ import annotations

import numpy as np


def softplus(nu):
    return np.logaddexp(0.0, np.asarray(nu, np.float64))


def softplus_inv(theta):
    theta = np.asarray(theta, np.float64)
    return theta + np.log(-np.expm1(-theta))


def sigmoid(nu):
    nu = np.asarray(nu, np.float64)
    e = np.exp(-np.abs(nu))
    return np.where(nu >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def to_theta(nu, transform):
    return softplus(nu) if transform == "softplus" else np.exp(np.asarray(nu, np.float64))


def to_nu(theta, transform):
    return softplus_inv(theta) if transform == "softplus" else np.log(np.asarray(theta, np.float64))


def dtheta_dnu(nu, transform):
    return sigmoid(nu) if transform == "softplus" else np.exp(np.asarray(nu, np.float64))


class Adam:
    """Adam ascent on nu (maximising the marginal likelihood)."""

    def __init__(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = None
        self.v = None
        self.t = 0

    def step(self, nu, grad):
        grad = np.asarray(grad, np.float64)
        if self.m is None:
            self.m = np.zeros_like(grad)
            self.v = np.zeros_like(grad)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return np.asarray(nu, np.float64) + self.lr * mhat / (np.sqrt(vhat) + self.eps)
