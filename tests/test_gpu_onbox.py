"""The measured-ceiling kernels (matrix instructions only; a read-only
stream) through the C ABI: they run, report the operation count their
launch geometry implies, reach a plausible fraction of the datasheet peaks,
and reject bad arguments."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import paper_1412_1127_amd as ax
    ax.acc_init(0, 0)
    yield ax
    ax.acc_shutdown()


def _ms(torch, fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


@pytest.mark.parametrize("kind,per_inst,datasheet", [(0, 32 * 32 * 16 * 2, 2.5e15), (1, 32 * 32 * 32 * 2, 5.0e15)])
def test_mfma_loop(ax, kind, per_inst, datasheet):
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    s = torch.cuda.current_stream()
    print("onbox mfma kind=%d" % kind, flush=True)
    ops = ax.accx_onbox_mfma(kind, 2000, s)
    assert ops == cus * 8 * 2000 * 8 * per_inst
    rate = ops / (_ms(torch, lambda: ax.accx_onbox_mfma(kind, 2000, s)) * 1e-3)
    assert 0.3 * datasheet < rate <= 1.05 * datasheet


def test_read_stream(ax):
    import torch
    x = torch.ones(1 << 26, dtype=torch.float32, device="cuda")   # 256 MiB
    s = torch.cuda.current_stream()
    print("onbox read", flush=True)
    rate = x.numel() * 4 / (_ms(torch, lambda: ax.accx_onbox_read(x, x.numel() * 4, s), 5) * 1e-3)
    assert 1e12 < rate <= 9e12


def test_bad_arguments(ax):
    import torch
    x = torch.ones(64, dtype=torch.float32, device="cuda")
    for args in [(2, 10), (0, 0), (1, (1 << 30) + 1)]:
        with pytest.raises(ax.AccxError) as e:
            ax.accx_onbox_mfma(*args)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG
    for nbytes in (0, 12, -16):
        with pytest.raises(ax.AccxError) as e:
            ax.accx_onbox_read(x, nbytes)
        assert e.value.status == ax.ACC_ERR_INVALID_ARG
    with pytest.raises(ax.AccxError) as e:
        ax.accx_onbox_read(x.data_ptr() + 4, 16)
    assert e.value.status == ax.ACC_ERR_INVALID_ARG
