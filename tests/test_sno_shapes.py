"""Host-only validation of the surrogate's launch extents (no GPU needed).

With QHD_SNO_VALIDATE_ONLY=1 the library allocates nothing and launches
nothing: it walks the whole forward and backward sequence and checks, for every
GEMM operand and elementwise launch, that the extents the kernel will touch lie
inside one of its own buffers.  This runs every shape the GPU tests and the
benchmark use (and the edge cases of the descriptor's ranges) on the CPU before
any of them reaches a device."""
import pytest

from paper_2303_01471_amd import qhd as q

FAKE = 0x1000  # never dereferenced in validation mode


@pytest.fixture(autouse=True)
def _validate_only(monkeypatch):
    monkeypatch.setenv("QHD_SNO_VALIDATE_ONLY", "1")
    q.load_library()


SHAPES = [
    # (S, C, M, L, max_batch, batches)
    (32, 8, 4, 2, 8, (1, 3, 8)),
    (64, 16, 8, 1, 3, (1, 2, 3)),
    (128, 32, 16, 4, 4, (1, 2, 4)),
    (128, 32, 16, 4, 64, (64, 17)),
    (128, 32, 16, 4, 4096, (4096, 1000)),
    (32, 8, 16, 1, 2, (1, 2)),        # M = S/2
    (32, 64, 1, 3, 5, (5,)),          # one mode, widest channel count
    (256, 64, 32, 2, 2, (1, 2)),
    (64, 8, 5, 2, 7, (7, 3)),         # odd mode count
    # width 32 with 16 modes at every grid (the fused inference passes), and 8 modes
    (32, 32, 16, 2, 4, (4, 1)),
    (64, 32, 16, 2, 5, (5, 2)),
    (256, 32, 16, 2, 2, (2, 1)),
    (64, 32, 8, 2, 2, (2,)),
]


@pytest.mark.parametrize("S,C,M,L,Bmax,batches", SHAPES)
@pytest.mark.parametrize("precision", [q.QHD_SNO_BF16, q.QHD_SNO_FP32])
@pytest.mark.parametrize("train", [0, 1])
def test_every_launch_stays_inside_its_buffers(S, C, M, L, Bmax, batches, precision, train):
    h = q.qhd_sno_create(q.qhd_sno_desc(S, C, M, L, Bmax, precision, train, 3))
    try:
        for b in batches:
            q.qhd_sno_forward(h, FAKE, b, FAKE, 0)
            if train:
                q.qhd_sno_backward(h, FAKE, FAKE, b, 0, 0)
                q.qhd_sno_step(h, 1e-3, 0)
    finally:
        q.qhd_sno_destroy(h)


def test_parameter_count_matches_layout():
    from oracle import sno_reference as ref
    for S, C, M, L, *_ in SHAPES:
        h = q.qhd_sno_create(q.qhd_sno_desc(S, C, M, L, 1, q.QHD_SNO_BF16, 0, 0))
        try:
            assert q.qhd_sno_param_count(h) == ref.param_count(ref.Config(S=S, C=C, M=M, L=L))
        finally:
            q.qhd_sno_destroy(h)


def test_production_parameter_count():
    # width 32, 16 modes per axis, 4 layers: about 4.2 million parameters
    h = q.qhd_sno_create(q.qhd_sno_desc(128, 32, 16, 4, 1, q.QHD_SNO_BF16, 0, 0))
    try:
        n = q.qhd_sno_param_count(h)
    finally:
        q.qhd_sno_destroy(h)
    assert n == 32 * 3 + 32 + 4 * (2 * 32 * 16 * 32 * 32 + 32 * 32 + 32) + 32 + 1
    assert 4.1e6 < n < 4.3e6


@pytest.mark.parametrize("field,value", [("grid", 48), ("grid", 512), ("width", 24), ("width", 128),
                                         ("modes", 0), ("modes", 65), ("layers", 0), ("layers", 9),
                                         ("max_batch", 0), ("precision", 7)])
def test_invalid_descriptor_rejected(field, value):
    d = q.qhd_sno_desc(128, 32, 16, 4, 4, q.QHD_SNO_BF16, 1, 0)
    setattr(d, field, value)
    with pytest.raises(q.QHDError) as e:
        q.qhd_sno_create(d)
    assert e.value.status == q.QHD_EINVAL


def test_backward_needs_training_handle_and_step_needs_gradient():
    h = q.qhd_sno_create(q.qhd_sno_desc(32, 8, 4, 1, 2, q.QHD_SNO_BF16, 0, 0))
    try:
        with pytest.raises(q.QHDError) as e:
            q.qhd_sno_backward(h, FAKE, FAKE, 1, 0, 0)
        assert e.value.status == q.QHD_ESTATE
        with pytest.raises(q.QHDError) as e:
            q.qhd_sno_step(h, 1e-3, 0)
        assert e.value.status == q.QHD_ESTATE
        with pytest.raises(q.QHDError) as e:
            q.qhd_sno_forward(h, FAKE, 3, FAKE, 0)
        assert e.value.status == q.QHD_EINVAL
    finally:
        q.qhd_sno_destroy(h)
