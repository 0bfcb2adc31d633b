"""Host-side arithmetic of bench.py: the byte models it reports against."""
import bench


def test_pass_byte_model_values():
    # p (6 P s + 2 c) + c - 2 s with P = ceil(n / kmax): 888 B/amp at the headline
    # configuration (n = 32, p = 3, complex128), 1224 at n = 26, p = 6, 444 for complex64
    assert bench.model_bytes_per_amp(32, 3, 16, 8) == 888
    assert bench.model_bytes_per_amp(26, 6, 16, 8) == 1224
    assert bench.model_bytes_per_amp(32, 3, 8, 4) == 444


def test_batch_byte_model_counts_sweeps():
    # n <= 12: one sweep per layer; p = 4: forward 24 + 3 x 40, E/lam sweep 40,
    # backward 40 + 3 x 72
    assert bench.batch_bytes_per_amp(12, 4) == 24 + 3 * 40 + 40 + 40 + 3 * 72
    # two sweeps per layer with boundary sweeps: forward 24 + 3 x 40 + 1 x 32,
    # E/lam 40, backward 40 + 3 x 72 + 1 x 64
    assert bench.batch_bytes_per_amp(20, 4) == 24 + 3 * 40 + 32 + 40 + 40 + 3 * 72 + 64


def test_gpu_count_guard(capsys):
    import sys
    argv = sys.argv
    try:
        sys.argv = ["bench.py", "--gpus", "2"]
        assert bench.main() == 2
    finally:
        sys.argv = argv
    assert "one MI355X" in capsys.readouterr().err
