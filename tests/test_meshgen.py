"""The seeded generators: block-wise generation of large sets gives the same
arrays as one pass, and the sets have the documented structure."""
import numpy as np

import meshgen as mg


def _arrays(ms):
    return [ms.verts, ms.vert_begin, ms.vert_count, ms.tris, ms.tri_begin, ms.tri_count, ms.parent]


def test_blob_blocks_do_not_change_arrays(monkeypatch):
    a = mg.blob_set(mg.rng_for(9, 0), 37, (0.0, 50.0), 1, 3, radius_sigma=0.3)
    monkeypatch.setattr(mg, "BLOB_BLOCK_VALUES", 3 * 642)  # 3 blobs (642 finest vertices) per block
    b = mg.blob_set(mg.rng_for(9, 0), 37, (0.0, 50.0), 1, 3, radius_sigma=0.3)
    assert all(np.array_equal(x, y) for x, y in zip(_arrays(a), _arrays(b)))


def test_tube_blocks_do_not_change_arrays(monkeypatch):
    a = mg.tube_set(mg.rng_for(9, 1), 23, (0.0, 50.0), 64, 3)
    monkeypatch.setattr(mg, "TUBE_BLOCK", 5)
    b = mg.tube_set(mg.rng_for(9, 1), 23, (0.0, 50.0), 64, 3)
    assert all(np.array_equal(x, y) for x, y in zip(_arrays(a), _arrays(b)))


def test_worker_processes_and_threads_give_one_pass_arrays(monkeypatch):
    """Large sets are built in blocks by forked workers, or by threads of the
    process once it has opened the GPU; both write the same arrays as one
    serial pass."""
    monkeypatch.setattr(mg, "BLOB_BLOCK_VALUES", 3 * 642)
    monkeypatch.setattr(mg, "TUBE_BLOCK", 5)
    ref_b = mg.blob_set(mg.rng_for(9, 0), 37, (0.0, 50.0), 1, 3, radius_sigma=0.3, workers=1)
    ref_t = mg.tube_set(mg.rng_for(9, 1), 23, (0.0, 50.0), 64, 3, workers=1)
    for opened in (False, True):
        monkeypatch.setattr(mg, "_gpu_opened", lambda: opened)
        b = mg.blob_set(mg.rng_for(9, 0), 37, (0.0, 50.0), 1, 3, radius_sigma=0.3, workers=4)
        t = mg.tube_set(mg.rng_for(9, 1), 23, (0.0, 50.0), 64, 3, workers=4)
        assert all(np.array_equal(x, y) for x, y in zip(_arrays(ref_b), _arrays(b))), opened
        assert all(np.array_equal(x, y) for x, y in zip(_arrays(ref_t), _arrays(t))), opened


def test_multilod_structure():
    R, S = mg.config_multilod(seed=1, n_r=7, n_s=3, box=50.0, n_seg=64)
    assert R.n_lods == S.n_lods == 4
    assert R.tri_count.reshape(7, 4).tolist() == [[80, 320, 1280, 5120]] * 7
    # tubes: 16 triangles per segment plus two 8-triangle caps, segments / 4 per coarser LoD
    assert S.tri_count.reshape(3, 4).tolist() == [[16 * 1 + 16, 16 * 4 + 16, 16 * 16 + 16, 16 * 64 + 16]] * 3
    # every object's boxes fit inside the scene box, up to its own size
    for ms in (R, S):
        for o in range(ms.n_objects):
            v = ms.verts[ms.vert_begin[o]:ms.vert_begin[o] + ms.vert_count[o]]
            c = 0.5 * (v.min(0) + v.max(0))
            assert np.all(c >= -1e-3) and np.all(c <= 50.0 + 1e-3)


def test_worker_processes_do_not_change_arrays(monkeypatch):
    """The large sets are built by forked workers into shared memory (blob
    noise from a generator advanced past the earlier blocks); the arrays are
    those of one serial pass."""
    monkeypatch.setattr(mg, "BLOB_BLOCK_VALUES", 4 * 2562)
    monkeypatch.setattr(mg, "TUBE_BLOCK", 3)
    a = mg.config_large(n_r=41, n_s=10, box=300.0, n_seg=64, workers=1)
    b = mg.config_large(n_r=41, n_s=10, box=300.0, n_seg=64, workers=3)
    for x, y in zip(a, b):
        assert all(np.array_equal(p, q) for p, q in zip(_arrays(x), _arrays(y)))
