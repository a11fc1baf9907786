"""The byte accounting behind bench.py's roofline figures, against sums written
out by hand for the 256^3, R = 10 workload (no GPU needed).

Algorithmic bytes of one MTTKRP: the tensor once (P b), the other factors
(sum_{m != n} I_m R b) and the I_n x R FP64 output.  With the dimension tree
the mode-1 launch also writes the stage-1 tiles Y (S I_1 R entries in the
tensor's precision; reported as overhead) and the modes >= 2 read Y instead of
the tensor, with the FP64 factors of the modes >= 1 other than n."""
import bench

DIMS, R = (256, 256, 256), 10


def test_plain_mttkrp_bytes():
    P = 256 ** 3
    assert bench.mttkrp_bytes(DIMS, R, 0, 4) == P * 4 + 2 * 256 * R * 4 + 256 * R * 8 == 67149824
    assert bench.mttkrp_bytes(DIMS, R, 2, 8) == P * 8 + 2 * 256 * R * 8 + 256 * R * 8


def test_dimension_tree_bytes_fp32_and_fp64():
    y = 256 * 256 * R   # S I1 R entries
    assert bench.tree_y_doubles(DIMS, R, 4) == y
    # mode 0 streams Z as usual; mode 1 also stores Y (overhead), modes >= 2 read Y
    assert bench.sweep_mttkrp_bytes(DIMS, R, 0, 4) == bench.mttkrp_bytes(DIMS, R, 0, 4)
    assert bench.sweep_mttkrp_overhead_bytes(DIMS, R, 1, 4) == y * 4 == 2621440
    assert bench.sweep_mttkrp_overhead_bytes(DIMS, R, 1, 8) == y * 8 == 5242880
    assert bench.sweep_mttkrp_overhead_bytes(DIMS, R, 2, 4) == 0
    assert bench.sweep_mttkrp_bytes(DIMS, R, 2, 4) == y * 4 + 256 * R * 8 + 256 * R * 8
    assert bench.sweep_mttkrp_bytes(DIMS, R, 2, 8) == y * 8 + 256 * R * 8 + 256 * R * 8


def test_no_tree_cases():
    # order 2, and Y above a quarter of the tensor's bytes: one pass per mode
    assert bench.tree_y_doubles((300, 200), 5, 8) == 0
    assert bench.tree_y_doubles((4, 64, 64), 10, 8) == 0   # Y = 64*64*10*8 B > (4*64*64*8) / 4 B
    assert bench.sweep_mttkrp_bytes((4, 64, 64), 10, 2, 8) == bench.mttkrp_bytes((4, 64, 64), 10, 2, 8)


def test_batched_tile_choice_prefers_the_smaller_tile_on_a_near_tie():
    """The batched tile tuner times the batch with every restart active; on a
    near tie (within 3 %) the smaller tile wins, otherwise the fastest."""
    from paper_1111_6091_amd.drivers import pick_tile
    # measured: 96 KiB 16.56 ms against 192 KiB 16.43 ms (mixed) -> 96
    assert pick_tile({48: 24.17, 96: 16.56, 192: 16.43, 384: 17.44, 768: 19.15}) == 96
    # 96 KiB 4 % slower than 192 KiB (FP64) -> 192
    assert pick_tile({48: 19.45, 96: 17.05, 192: 16.39, 384: 16.63, 768: 17.78}) == 192
    assert pick_tile({48: 1.0}) == 48
    assert pick_tile({48: 2.0, 96: 1.0}, near=0.0) == 96
