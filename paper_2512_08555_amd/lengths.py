"""Padded FFT lengths the compiled kernels cover."""
from . import _capi as capi


def supported_length(m, prec="f64"):
    return bool(capi.lib().ups_supported_length(int(m), capi.UPS_F64 if prec == "f64" else capi.UPS_F32))


def auto_pad(shape, prec="f64"):
    """Smallest supported padded length >= 2 n per axis for a (nz, ny, nx)
    grid (the kernels need M >= 2 n; see include/ups.h)."""
    out = []
    for n in shape:
        m = 2 * int(n)
        while not supported_length(m, prec):
            m += 2
            if m > 16384:
                raise ValueError("no supported padded length for n = %d" % n)
        out.append(m)
    return tuple(out)
