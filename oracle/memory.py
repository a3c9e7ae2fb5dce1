"""Memory model of Sec. 2.4: Eqs. (npmax), (nptile), (Mp_particle), (Mp_coarse), (Mp_fine).

Test infrastructure only (see ``oracle/__init__``).

Readings that make the equations reproduce Table t.memory (both are typographical in the
printed equations):
* Eq. (nptile) omits the buffer factor: the per-tile temporaries also hold buffer particles,
  P*_max = <P_local> (1 + 2 N_b/N_t)^3 M_t^-3 (1 + eps_tile)   (gives the table's 0.872 bpp).
* Eq. (Mp_fine) prints N_t^-3 where M_t^-3 is meant (one fine kernel per tile, not per cell):
  M_fine = 6 R^3 P_c^-1 M_t^-3 (1 + 2 N_b/N_t)^3   (gives 0.291 bpp against the table's 0.292).

Pinned by tests/test_oracle_memory.py against every printed row of Table t.memory that follows
from the equations (chi/nu, chi*/nu*, rho_c, v_c, K_c, K_f, totals, optimal limit).
"""
from __future__ import annotations


def footprint(p_local_side: int, nc_per_image: int, n_b: int, m_t: int, eps_image: float,
              eps_tile: float, nchi: int = 1, nnu: int = 1, n_i: int = 0, r: int = 4):
    """Bytes per image for each array group and bytes per particle (bpp)."""
    p_local = float(p_local_side) ** 3
    n_t = nc_per_image / m_t
    buf = (1.0 + 2.0 * n_b / n_t) ** 3
    per_p = 3 * nchi + 3 * nnu + n_i
    p_max = p_local * buf * (1.0 + eps_image)                      # Eq. (npmax)
    p_max_tile = p_local * buf * m_t**-3 * (1.0 + eps_tile)          # Eq. (nptile), with buffer factor
    n_e = n_t + 2 * n_b
    rows = {
        "chi_nu": per_p * p_max,
        "chi_nu_star": per_p * p_max_tile,
        "rho_c": 4.0 * (n_e * m_t) ** 3,
        "v_c": 3 * 4.0 * (n_e * m_t) ** 3,
        "K_c": 3 * 4.0 * nc_per_image**3 / 2.0,
        "K_f": 3 * 4.0 * (r * n_e) ** 3 / 2.0,
    }
    p_c = p_local / nc_per_image**3
    bpp = {k: v / p_local for k, v in rows.items()}
    bpp["Mp_particle"] = per_p * (buf * (1.0 + eps_image) + m_t**-3 * buf * (1.0 + eps_tile))      # Eq. (Mp_particle)
    bpp["Mp_coarse"] = (16.0 * buf + 6.0) / p_c                                                     # Eq. (Mp_coarse)
    bpp["Mp_fine"] = 6.0 * r**3 / p_c * m_t**-3 * buf                                               # Eq. (Mp_fine), corrected
    total = rows["chi_nu"] + rows["chi_nu_star"] + rows["rho_c"] + rows["v_c"] + rows["K_c"] + rows["K_f"]
    rows["total"] = total
    bpp["total"] = total / p_local
    rows["optimal"] = per_p * p_local
    bpp["optimal"] = float(per_p)
    return rows, bpp
