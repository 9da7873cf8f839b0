"""Host-side pieces of the network's training driver (CPU only): parameter
initialisation in the library's layout and checkpoint round trips."""
import numpy as np
import pytest

gp = pytest.importorskip("paper_1710_08231_amd")
torch = pytest.importorskip("torch")


def _lib_or_skip():
    try:
        gp.load()
    except gp.GPError:
        pytest.skip("libgp.so not built")


def test_init_params_layout():
    _lib_or_skip()
    from paper_1710_08231_amd import train_mpnn
    w = train_mpnn.init_params(16, seed=3)
    assert w.dtype == np.float32 and w.size == gp.mpnn_param_count(16) == 19920
    # biases (64 after each layer's two matrices, k at the end) start at zero
    o = 0
    for din in (18, 64, 64):
        o += 2 * 64 * din
        assert np.all(w[o:o + 64] == 0)
        o += 64
    assert np.all(w[-16:] == 0)
    assert np.array_equal(w, train_mpnn.init_params(16, seed=3))


def test_checkpoint_round_trip(tmp_path):
    _lib_or_skip()
    from paper_1710_08231_amd import train_mpnn
    P = gp.mpnn_param_count(8)
    rng = np.random.default_rng(0)
    w, m, v = (torch.from_numpy(rng.normal(0, 1, P).astype(np.float32)) for _ in range(3))
    path = str(tmp_path / "ck.npz")
    train_mpnn.save_checkpoint(path, w, m, v, step=1234, cursor=567)
    w2, m2, v2, step, cursor = train_mpnn.load_checkpoint(path)
    assert np.array_equal(w2, w.numpy()) and np.array_equal(m2, m.numpy()) and np.array_equal(v2, v.numpy())
    assert (step, cursor) == (1234, 567)


def test_committed_weights_match_layout():
    _lib_or_skip()
    import os
    path = os.path.join(os.path.dirname(gp.__file__), "mpnn_k16.npy")
    w = np.load(path)
    assert w.dtype == np.float32 and w.size == gp.mpnn_param_count(16)
    assert np.all(np.isfinite(w))
