"""The FP64 oracle on several host threads: one oracle call per wavelength, run concurrently
(numpy's transforms and elementwise kernels release the interpreter lock), results gathered
in wavelength order.  Test infrastructure, like the oracle itself; nothing here computes the
method, it only spreads the oracle's own per-wavelength calls over the host cores."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import dpx_oracle as o


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _map(fn, items):
    with ThreadPoolExecutor(max_workers=workers()) as ex:
        return list(ex.map(fn, items))


def forward(design, h, u_in, wavelengths, mode="fft"):
    """o.forward over the listed wavelengths: [len(wavelengths), T, T]."""
    return np.concatenate(_map(lambda w: o.forward(design, h, u_in, mode, wavelengths=[w]), wavelengths))


def grad(design, h, u_in, dl_di, wavelengths, mode="fft"):
    """o.grad over the listed wavelengths (dl_di[i] belongs to wavelengths[i]), summed in the
    order of the list."""
    parts = _map(lambda i: o.grad(design, h, u_in, dl_di[i:i + 1], mode, wavelengths=[wavelengths[i]]),
                 range(len(wavelengths)))
    total = np.zeros_like(parts[0])
    for p in parts:
        total += p
    return total


def loss(design, h, u_in, tau, wavelengths, mode="fft"):
    """The loss over the listed wavelengths only (tau[i] belongs to wavelengths[i])."""
    return o.loss(forward(design, h, u_in, wavelengths, mode), tau)[0]
