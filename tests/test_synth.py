"""Seeded input generators: determinism and the structure the workloads state."""
import numpy as np

from paper_1909_10547_amd import synth


def test_config_sizes_and_determinism():
    c1, c2 = synth.dis_fit_workload(), synth.had_fit_workload()
    assert len(c1.ndata) == 20 and all(50 <= n <= 600 for n in c1.ndata)
    assert len(c2.ndata) == 10 and all(20 <= n <= 1000 for n in c2.ndata)
    assert synth.dis_fit_workload().ndata == c1.ndata
    c0 = synth.dis_single_workload()
    assert c0.ndata == [100] and c0.xgrid.shape == (30,) and c0.nrep == 1
    assert np.isclose(c0.xgrid[0], 1e-5) and np.isclose(c0.xgrid[-1], 0.9)
    assert np.isclose(c1.xgrid[0], 1e-7) and c1.xgrid[-1] == 1.0


def test_dis_masks_and_values():
    w = synth.dis_fit_workload(scale=0.05)
    t0 = w.table(3)
    t1 = w.table(3)
    np.testing.assert_array_equal(t0.fk, t1.fk)
    assert int(t0.mask.sum()) == 9 and t0.fk.shape == (w.ndata[3], 9, 50)


def test_had_masks_symmetry_and_counts():
    w = synth.had_fit_workload(scale=0.02)
    t = w.table(0)
    assert int(t.mask.sum()) == 60
    assert int(np.trace(t.mask)) == 4
    np.testing.assert_array_equal(t.mask, t.mask.T)
    pairs = synth.pair_list(t.mask)
    idx = {(int(a), int(b)): c for c, (a, b) in enumerate(pairs)}
    for (a, b), c in idx.items():
        np.testing.assert_array_equal(t.fk[:, c], np.transpose(t.fk[:, idx[(b, a)]], (0, 2, 1)))


def test_pdf_replicas():
    w = synth.dis_fit_workload(scale=0.05)
    f = w.pdf()
    assert f.shape == (14, 50, 100)
    assert np.all(np.isfinite(f))
    assert np.all(f[:, -1, :] == 0.0)          # x = 1 gives (1-x)^q = 0
    assert np.all(f[:, :-1, :] > 0)
    c = w.central_pdf()
    assert c.shape == (14, 50, 1)
    assert not np.allclose(f[:, :, 0], f[:, :, 1])   # replicas are jittered


def test_covariance_block_is_spd():
    rng = np.random.default_rng(0)
    C, D = synth.covariance_block(rng.normal(size=50), np.random.default_rng(1))
    assert np.allclose(C, C.T)
    assert np.min(np.linalg.eigvalsh(C)) > 0
    assert D.shape == (50,)
