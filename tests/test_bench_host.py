"""Host-side arithmetic of bench.py: the byte models it reports against."""
import bench


def test_pass_byte_model_values():
    # p (6 P s + 2 c) + c - 2 s with P = ceil(n / kmax): 888 B/amp at the headline
    # configuration (n = 32, p = 3, complex128), 1224 at n = 26, p = 6, 444 for complex64
    assert bench.model_bytes_per_amp(32, 3, 16, 8) == 888
    assert bench.model_bytes_per_amp(26, 6, 16, 8) == 1224
    assert bench.model_bytes_per_amp(32, 3, 8, 4) == 444


def test_batch_byte_model_counts_sweeps():
    # n <= 12: one sweep per layer; p = 4: forward 24 + 2 x 40 (layers 0..2), the
    # turn 40 (layer 3), backward 2 x 72 + 40 (layers 2..0)
    assert bench.batch_bytes_per_amp(12, 4) == 24 + 2 * 40 + 40 + 2 * 72 + 40
    # p = 1 at n <= 12: the turn generates the state and stores nothing, reading C only
    assert bench.batch_bytes_per_amp(12, 1) == 8
    # two sweeps per layer with boundary sweeps: forward 24 + 3 x 40, the turn 40,
    # backward 3 x 72 + 40 (the alternating group order leaves no plain sweep)
    assert bench.batch_bytes_per_amp(20, 4) == 24 + 3 * 40 + 40 + 3 * 72 + 40
    # three sweeps per layer (depth 4 at n = 20): one plain sweep per layer beyond
    # the boundary ones, each way: forward 24 + 3 x 40 + 4 x 32, backward + 4 x 64
    assert bench.batch_bytes_per_amp(20, 4, 4) == 24 + 3 * 40 + 4 * 32 + 40 + 3 * 72 + 40 + 4 * 64


def test_gpu_count_guard(capsys):
    import sys
    argv = sys.argv
    try:
        sys.argv = ["bench.py", "--gpus", "2"]
        assert bench.main() == 2
    finally:
        sys.argv = argv
    assert "one MI355X" in capsys.readouterr().err
