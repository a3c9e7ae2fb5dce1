"""Table t.memory (Sec. 2.4) reproduced from Eqs. (npmax)-(Mp_fine)."""
import pytest

from oracle.memory import footprint


def test_table_t_memory():
    rows, bpp = footprint(1536, 384, 6, 3, 0.05, 2.0)
    gb = {k: v / 1e9 for k, v in rows.items()}
    assert gb["chi_nu"] == pytest.approx(29.9, abs=0.05)
    assert bpp["chi_nu"] == pytest.approx(8.24, abs=0.005)
    assert gb["chi_nu_star"] == pytest.approx(3.16, abs=0.005)
    assert bpp["chi_nu_star"] == pytest.approx(0.872, abs=0.0005)
    assert gb["rho_c"] == pytest.approx(0.296, abs=0.0005)
    assert bpp["rho_c"] == pytest.approx(0.0818, abs=0.00005)
    assert gb["v_c"] == pytest.approx(0.889, abs=0.0005)
    assert bpp["v_c"] == pytest.approx(0.245, abs=0.0005)
    assert gb["K_c"] == pytest.approx(0.340, abs=0.0005)
    assert bpp["K_c"] == pytest.approx(0.0939, abs=0.0002)  # printed 0.0939; equation gives 0.09375
    assert gb["K_f"] == pytest.approx(1.06, abs=0.01)
    assert bpp["Mp_fine"] == pytest.approx(0.292, abs=0.002)
    assert gb["total"] == pytest.approx(35.6, abs=0.05)
    assert bpp["total"] == pytest.approx(9.84, abs=0.02)
    assert gb["optimal"] == pytest.approx(21.7, abs=0.05)
    assert rows["optimal"] / rows["total"] == pytest.approx(0.610, abs=0.002)
    # Eq. (Mp_particle) is the sum of the two particle rows
    assert bpp["Mp_particle"] == pytest.approx(bpp["chi_nu"] + bpp["chi_nu_star"], rel=1e-12)
    # Eq. (Mp_coarse) is the rho_c + v_c + K_c rows
    assert bpp["Mp_coarse"] == pytest.approx(bpp["rho_c"] + bpp["v_c"] + bpp["K_c"], rel=1e-12)
