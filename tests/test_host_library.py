"""Host side of libsaq.so (no GPU needed): the C ABI loads and exports every
declared symbol, and the plan fit (Sections 4.1-4.2) agrees with the oracle
and with LAPACK."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
import paper_2509_12086_amd as saq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "saq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(saq_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 18
    L = ctypes.CDLL(saq.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(saq.EXPORTS)
    assert b"gfx950" in saq.lib().saq_version()


def test_eigensolver_matches_lapack():
    """Library fit without segment rotation: M's rows are the kept
    eigenvectors and the stored variances the eigenvalues (descending)."""
    ds = synth.cfg1(4000)
    X = ds.rows()
    p = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=8.0, rotate_segments=False, fit_sample=0))
    M, c, var = p.arrays()
    mu, cov, lam, V = oracle.pca(X)
    assert np.allclose(c, mu.astype(np.float32), rtol=0, atol=1e-6)
    assert np.allclose(var, lam, rtol=1e-9, atol=1e-12 * lam[0])
    # eigenvectors up to sign, for well-separated eigenvalues
    gaps = np.minimum(np.abs(np.diff(lam, prepend=np.inf)), np.abs(np.diff(lam, append=-np.inf)))
    for j in range(p.D_kept):
        if gaps[j] > 1e-3 * lam[0]:
            assert abs(float(M[j].astype(np.float64) @ V[:, j])) == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("D,bpd", [(64, 2.0), (128, 4.0), (100, 3.0), (96, 0.5)])
def test_fit_against_oracle_plan(D, bpd):
    rng = np.random.default_rng(D)
    lam = np.sort(rng.gamma(0.7, 1.0, size=D))[::-1]
    R = synth.haar_rotation(D, 5)
    X = ((rng.standard_normal((3000, D)) * np.sqrt(lam)) @ R.T).astype(np.float32)
    params = saq.PlanParams(bits_per_dim=bpd, granularity=16, max_bits=9, max_width=64,
                            fit_sample=0, seed=3)
    p = saq.Plan.fit(X, params)
    _, _, var = p.arrays()
    ref = oracle.plan_search(var, bpd, g=16, max_bits=9, max_width=64)
    assert p.info["min_error"] == pytest.approx(ref.min_error, rel=1e-10)
    assert len(p.widths) == ref.nseg
    assert p.info["model_error"] == pytest.approx(ref.error, rel=1e-10)
    assert p.info["used_bits"] <= oracle.quota_bits(bpd, D)
    assert sum(p.widths) == D
    assert all(w <= 64 for w, b in zip(p.widths, p.bits) if b > 0)
    assert oracle.plan_error(var, p.widths, p.bits) == pytest.approx(p.info["model_error"], rel=1e-10)


def test_rotated_basis_is_orthonormal_and_spans_segments():
    """Section 4.1: a random orthonormal rotation inside each segment; the
    rows of M stay orthonormal and each segment's rows span the same PCA
    subspace as without rotation."""
    ds = synth.cfg1(3000)
    X = ds.rows()
    base = saq.PlanParams(bits_per_dim=4.0, fit_sample=0, seed=9)
    p_rot = saq.Plan.fit(X, base)
    p_raw = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0, rotate_segments=False))
    assert p_rot.widths == p_raw.widths and p_rot.bits == p_raw.bits
    Mr, _, _ = p_rot.arrays()
    M0, _, _ = p_raw.arrays()
    Mr64, M064 = Mr.astype(np.float64), M0.astype(np.float64)
    assert np.allclose(Mr64 @ Mr64.T, np.eye(p_rot.D_kept), atol=5e-6)
    off = 0
    for w in p_rot.kept_widths:
        Rs = Mr64[off:off + w] @ M064[off:off + w].T          # the segment's rotation
        assert np.allclose(Rs @ Rs.T, np.eye(w), atol=5e-6)
        assert np.abs(Rs - np.eye(w)).max() > 0.1            # actually rotated
        off += w
    # seeded: the same seed gives the same matrix, another seed another one
    assert np.array_equal(saq.Plan.fit(X, base).arrays()[0], Mr)
    other = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0, seed=10)).arrays()[0]
    assert not np.array_equal(other, Mr)


def test_uniform_spectrum_single_segment():
    D = 64
    p = saq.Plan.from_basis(np.zeros(D), np.eye(D), np.ones(D),
                            saq.PlanParams(bits_per_dim=3.0, max_width=0))
    assert p.widths == [64] and p.bits == [3]


def test_plan_save_load_roundtrip(tmp_path):
    X = synth.cfg1(2000).rows()
    p = saq.Plan.fit(X, saq.PlanParams(fit_sample=0))
    path = str(tmp_path / "p.saqplan")
    p.save(path)
    q = saq.Plan.load(path)
    assert q.widths == p.widths and q.bits == p.bits and q.info == p.info
    for a, b in zip(p.arrays(), q.arrays()):
        assert np.array_equal(a, b)
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0xFF
    bad = str(tmp_path / "bad.saqplan")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(saq.SaqError, match="SAQ_EIO"):
        saq.Plan.load(bad)
    open(bad, "wb").write(bytes(raw[:50]))
    with pytest.raises(saq.SaqError, match="SAQ_EIO"):
        saq.Plan.load(bad)
    with pytest.raises(saq.SaqError, match="SAQ_EIO"):
        saq.Plan.load(str(tmp_path / "missing"))


def _fnv1a(b: bytes) -> int:
    h = 0xcbf29ce484222325
    for x in b:
        h = ((h ^ x) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_plan_file_carries_the_spread_blocks(tmp_path):
    """The plan keeps, per kept segment, S_s = diag(sqrt(lambda)) R_s^T
    (Section 4.3's sigma_Seg from the query's projection).  Read back from the
    file: S_s S_s^T = diag(lambda) (R_s is orthonormal) and S_s M_s has
    orthogonal rows of norm sqrt(lambda) (M_s = R_s P_s).  A version-1 file,
    which has no blocks, still loads."""
    X = synth.cfg1(3000).rows()
    p = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0))
    path = str(tmp_path / "p.saqplan")
    p.save(path)
    raw = open(path, "rb").read()
    kw = p.kept_widths
    nS = int(sum(w * w for w in kw))
    tail = raw[len(raw) - 8 - 4 * nS - 8: len(raw) - 8]
    assert int(np.frombuffer(tail[:8], np.int64)[0]) == nS
    S = np.frombuffer(tail[8:], np.float32).astype(np.float64)
    M, _, var = p.arrays()
    lam_kept, pos = [], 0
    for w, b in zip(p.widths, p.bits):
        if b > 0:
            lam_kept.extend(var[pos:pos + w])
        pos += w
    lam_kept = np.asarray(lam_kept)
    a = r = 0
    for w in kw:
        Sb = S[a:a + w * w].reshape(w, w)
        lam = lam_kept[r:r + w]
        np.testing.assert_allclose(Sb @ Sb.T, np.diag(lam), rtol=0, atol=1e-5 * lam.max())
        SM = Sb @ M[r:r + w].astype(np.float64)
        np.testing.assert_allclose(SM @ SM.T, np.diag(lam), rtol=0, atol=1e-5 * lam.max())
        a += w * w
        r += w
    # version 1: the same file without the blocks
    body = bytearray(raw[:len(raw) - 8 - 4 * nS - 8])
    body[8:12] = np.uint32(1).tobytes()
    v1 = bytes(body) + np.uint64(_fnv1a(bytes(body))).tobytes()
    old = str(tmp_path / "v1.saqplan")
    open(old, "wb").write(v1)
    q = saq.Plan.load(old)
    assert q.widths == p.widths and q.bits == p.bits
    assert q.device_bytes() < p.device_bytes()


def test_from_parts_and_argument_errors():
    D = 32
    M = np.eye(D, dtype=np.float32)[:24]
    p = saq.Plan.from_parts([16, 8, 8], [4, 2, 0], M, np.zeros(D, np.float32))
    assert p.D_kept == 24 and p.code_bytes == 4 * 2 + 2 * 1 and p.n_factors == 3
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.Plan.from_parts([16, 8], [4, 2], M, np.zeros(D, np.float32))     # widths != D
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.Plan.from_parts([32], [17], np.eye(D, dtype=np.float32), np.zeros(D, np.float32))
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.Plan.fit(np.zeros((10, 8), np.float32), saq.PlanParams(granularity=0))
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.Plan.fit(np.zeros((10, 8), np.float32), saq.PlanParams(max_width=12, granularity=8))
    # device calls on a plan that was never uploaded are rejected on the host
    L = saq.lib()
    assert L.saq_encode(p._h, None, 10, 4, None, None, None, 0, None) == 1
    assert L.saq_quantize(p._h, None, 24, 0, 10, None, 4, None, None, None) == 1
    assert L.saq_encode_workspace_bytes(p._h, -1) == -1


def test_record_size_formula():
    """code_bytes = sum over kept segments of B * ceil(W/8)."""
    D = 40
    p = saq.Plan.from_parts([16, 12, 12], [9, 3, 1], np.eye(D, dtype=np.float32),
                            np.zeros(D, np.float32))
    assert p.code_bytes == 9 * 2 + 3 * 2 + 1 * 2
    assert p.kept_widths == [16, 12, 12] and p.kept_bits == [9, 3, 1]


def test_projection_accumulation_mode():
    """Auto mode adds the projection's k-tiles in FP64 for long inputs or
    fine grids (D > 1024 or a kept segment with >= 8 bits), else FP32."""
    def mode(D, bits, acc):
        M = np.eye(D, dtype=np.float32)[:16]
        p = saq.Plan.from_parts([16, D - 16], [bits, 0], M, np.zeros(D, np.float32))
        return p.info["projection_fp64_totals"]
    assert mode(960, 7, 0) == 0 and mode(960, 8, 0) == 1 and mode(2048, 4, 0) == 1
    X = np.random.default_rng(0).standard_normal((500, 64)).astype(np.float32)
    for acc, want in ((0, 0), (1, 0), (2, 1)):
        p = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=2.0, fit_sample=0, projection_accumulation=acc))
        assert p.info["projection_fp64_totals"] == want


def test_fit_is_independent_of_thread_count(tmp_path):
    """The host fit gives bit-identical plans for any OpenMP thread count (its
    reductions run over fixed row blocks in a fixed order)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r)\n"
        "import synth, paper_2509_12086_amd as saq\n"
        "X = synth.cfg1(9000).rows()\n"
        "saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).save(sys.argv[1])\n"
    ) % root
    paths = []
    for threads in (1, 5):
        out = str(tmp_path / f"plan_{threads}.saq")
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        subprocess.run([sys.executable, "-c", code, out], env=env, check=True, timeout=300)
        paths.append(out)
    a, b = (saq.Plan.load(p_) for p_ in paths)
    for x, y in zip(a.arrays(), b.arrays()):
        assert np.array_equal(x, y)
    assert a.widths == b.widths and a.bits == b.bits
