"""The seeded input generators: the device-side jet labels equal the host ones bit for bit, and
the labelled assembly is a pure selection of the given states."""
import numpy as np
import torch

import workloads as W


def test_jet_patch_list_shape_and_levels():
    pl = W.jet_patch_list(n_patch=20_000, n_base=128)
    lv = pl["level"]
    assert pl["corner"].shape == (20_000, 3) and lv.dtype == np.int8
    counts = np.bincount(lv, minlength=4)
    assert np.array_equal(counts, [1000, 2000, 5000, 12000])
    # every patch lies inside its level's lattice, no patch is listed twice
    npl = (128 << lv.astype(np.int64)) // 8
    assert np.all(pl["corner"] >= 0) and np.all(pl["corner"] // 8 < npl[:, None])
    key = np.concatenate([lv[:, None].astype(np.int64), pl["corner"]], axis=1)
    assert np.unique(key, axis=0).shape[0] == key.shape[0]
    try:
        W.jet_patch_list(n_patch=20_000, n_base=64)      # level 0 has only 512 patches
    except ValueError:
        pass
    else:
        raise AssertionError("an over-full level must be rejected")


def test_jet_labels_torch_equal_numpy():
    pl = W.jet_patch_list(n_patch=4000, n_base=64, r_jet=0.05, z_jet=0.1)
    a = W.jet_labels(pl)
    b = W.jet_labels_torch(pl, "cpu", chunk=1000).numpy()
    assert a.any() and not a.all()
    assert np.array_equal(a, b)


def test_assemble_labeled_is_a_selection():
    rng = np.random.default_rng(3)
    lab = rng.integers(0, 2, (7, 14, 14, 14)).astype(np.uint8)
    st = rng.standard_normal((2, 5))
    x = W.assemble_labeled(lab, st)
    y = W.assemble_labeled(torch.from_numpy(lab), st).numpy()
    assert x.shape == (7, 5, 14, 14, 14)
    assert np.array_equal(x, y)
    for f in range(5):
        assert np.array_equal(x[:, f], np.where(lab == 1, st[1, f], st[0, f]))
