"""Choosing the grid resolution for a flux error threshold.

The interpolated model's accuracy is set by its discretisation: the number
of annuli (inside and outside z_cut, Sect. 3.1.1) and of grazing values
(Sect. 3.1.2).  The paper chooses them from its accuracy figure (Sect. 3.3);
``tune_grid`` chooses them, and the inner/limb division z_cut, for a given
profile and error threshold: for each z_cut it walks a ladder of (nzin,
nzlimb, ng) from coarse to fine to the first level whose fluxes, over probe
separations z in [0, 1 + k) and probe radius ratios, stay within the
threshold of a much finer reference grid, and returns the cheapest of
those.  Every
flux is computed by the library (rr_flux_at_z); each probe k is made a node
of its own two-node k-grid, so the k-interpolation does not enter (its
contribution is set by nk separately).
"""

import numpy as np

from .api import Tables, flux_at_z

# (nzin, nzlimb, ng): coarse to fine
LADDER = ((10, 20, 64), (15, 30, 100), (20, 40, 128), (30, 60, 192), (40, 80, 256),
          (60, 120, 512), (90, 180, 768), (120, 240, 1024))
REFERENCE = (400, 800, 2048)


def _probe_z(k, n):
    """Separations over [0, 1 + k), denser across the limb contacts."""
    zs = np.concatenate([np.linspace(0.0, 1.0 + k, n, endpoint=False),
                         np.linspace(max(0.0, 1.0 - k), 1.0 + k, n, endpoint=False)])
    return np.unique(zs)


def _fluxes(mu, prof, level, ks, zs, zcut, precision):
    out = []
    for k, z in zip(ks, zs):
        grid = dict(zcut=zcut, nzin=level[0], nzlimb=level[1], ng=level[2], nk=2,
                    k0=float(k), k1=float(k) + 1e-3)
        tab = Tables(mu, prof, grid)
        out.append(flux_at_z(tab, z, float(k), 0, precision).cpu().numpy().astype(np.float64))
        tab.close()
    return out


def tune_grid(mu, prof, max_err_ppm, k_range=(0.01, 0.3), zcut=None,
              zcuts=(0.5, 0.6, 0.7, 0.8, 0.9), nprobe_k=6, nprobe_z=400, ladder=LADDER,
              reference=REFERENCE, precision="fp64"):
    """The cheapest grid whose flux error against the reference grid is at
    most ``max_err_ppm`` (parts per million of the stellar flux) for the
    single profile ``prof`` sampled at ``mu``: the inner/limb division z_cut
    (each of ``zcuts``, or only ``zcut`` if given) and the resolutions
    (nzin, nzlimb, ng) of a ladder level are chosen together (Sect. 3.1.1:
    both are tuned for a profile and an error threshold).  For every z_cut
    the ladder is walked from coarse to fine up to the first level within
    the threshold; of those, the grid with the fewest weight entries
    (nz x ng, the cost of building and holding the weights) wins, the
    smaller error breaking ties.  Returns a dict with the chosen grid values
    (zcut, nzin, nzlimb, ng), its measured error and every (zcut, level)
    tried; ``grid`` is None if none meets the threshold."""
    ks = np.linspace(k_range[0], k_range[1], nprobe_k)
    zs = [_probe_z(k, nprobe_z) for k in ks]
    ref = _fluxes(mu, prof, reference, ks, zs, 0.8, "fp64")
    tried, best = [], None
    for zc in ((zcut,) if zcut is not None else zcuts):
        for level in ladder:
            f = _fluxes(mu, prof, level, ks, zs, zc, precision)
            err = max(float(np.abs(a - b).max()) for a, b in zip(f, ref)) * 1e6
            entry = dict(zcut=float(zc), nzin=level[0], nzlimb=level[1], ng=level[2],
                         max_err_ppm=err, cost=(level[0] + level[1]) * level[2])
            tried.append(entry)
            if err <= max_err_ppm:
                if best is None or (entry["cost"], err) < (best["cost"], best["max_err_ppm"]):
                    best = entry
                break
    if best is None:
        return dict(grid=None, max_err_ppm=None, tried=tried)
    return dict(grid=dict(zcut=best["zcut"], nzin=best["nzin"], nzlimb=best["nzlimb"],
                          ng=best["ng"]), max_err_ppm=best["max_err_ppm"], tried=tried)


def probe_errors(mu, prof, level, ks, zs, exact, zcut=0.8, precision="fp64"):
    """Flux errors of one grid level against exact fluxes ``exact[i]`` at
    separations ``zs[i]`` and radius ratios ``ks[i]`` (for accuracy studies
    such as the paper's error-versus-grazing figure)."""
    f = _fluxes(mu, prof, level, ks, zs, zcut, precision)
    return [a - np.asarray(e, float) for a, e in zip(f, exact)]


__all__ = ["tune_grid", "probe_errors", "LADDER", "REFERENCE"]
