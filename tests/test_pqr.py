"""The PQR reader: records with and without a chain identifier, other records skipped,
malformed records rejected, and a write/read round trip of a synthetic molecule."""
import numpy as np
import pytest

from paper_1709_08070_amd import pqr, synth


def test_reads_the_fixture(tmp_path):
    import os

    atoms = pqr.read_pqr(os.path.join(os.path.dirname(__file__), "golden", "synthetic_small.pqr"))
    want = np.array([[-1.2, 0.0, 0.0, 1.6, -0.5], [1.2, 0.0, 0.0, 1.6, 0.5], [0.0, 1.8, 0.4, 1.2, 1.0],
                     [0.0, -1.7, -0.3, 1.5, -1.0]])
    np.testing.assert_array_equal(atoms, want)
    assert atoms[:, 4].sum() == 0.0


def test_round_trip(tmp_path):
    atoms = synth.globule(60, 3)
    path = str(tmp_path / "g.pqr")
    pqr.write_pqr(path, atoms)
    back = pqr.read_pqr(path)
    np.testing.assert_allclose(back[:, :3], atoms[:, :3], atol=5e-4)
    np.testing.assert_allclose(back[:, 3], atoms[:, 3], atol=5e-5)
    np.testing.assert_allclose(back[:, 4], atoms[:, 4], atol=5e-5)


@pytest.mark.parametrize("line", ["ATOM      1  X1  MOL A   1      -1.200   0.000   0.000 -0.5000\n",
                                  "ATOM      1  X1  MOL A   1      -1.200   0.000   0.000 -0.5000 -1.0\n",
                                  "ATOM      1  X1  MOL A   1      -1.200   nan   0.000 -0.5000 1.0\n",
                                  "REMARK only\n"])
def test_rejects_malformed(tmp_path, line):
    path = tmp_path / "bad.pqr"
    path.write_text(line)
    with pytest.raises(ValueError):
        pqr.read_pqr(str(path))
