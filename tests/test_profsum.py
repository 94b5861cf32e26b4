"""Host-side bookkeeping of the measurement: the kernel names and workgroup
counts that bench.py and the profile summaries use to pick a kernel out of a
rocprofv3 trace must be the ones the library launches.  The expected values
are the names and grid sizes of the 513^3 FP32-in-FP64 solve's finest-level
kernels as they appear in its kernel trace (profiles/), and tile arithmetic
worked by hand: ceil(511 / tile width) x ceil(511 / tile rows) x z-chunks."""

from paper_1406_5369_amd import profsum


def test_pass_blocks_paired_and_single():
    # two nodes per lane: 128 nodes per tile row -> 4 x-tiles; 14 rows -> 37; 64 planes -> 8
    assert profsum.pass_blocks(3, 513, 16, 64, pairs=1) == 4 * 37 * 8 == 1184
    # one node per lane: 62 nodes per tile row -> 9 x-tiles; 30 rows -> 18; 32 planes -> 16
    assert profsum.pass_blocks(3, 513, 32, 32) == 9 * 18 * 16
    # 2D: 62 x 14 LDS tiles; with pairs, 128-node strips in 32-row chunks, four per workgroup
    assert profsum.pass_blocks(2, 4097, 16, 0) == 67 * 293
    assert profsum.pass_blocks(2, 4097, 16, 32, pairs=1) == 32 * 32
    assert profsum.pass_blocks(2, 1025, 16, 32, pairs=1) == 8 * 8
    # smallest grid: one tile
    assert profsum.pass_blocks(3, 5, 8, 1, pairs=1) == 1 * 1 * 3


def test_sweep_blocks():
    # two-node halo: 60 x 12 tiles of the 16-row box -> 9 x 43, 16-plane chunks -> 32
    assert profsum.sweep_blocks(3, 513, 16, 16) == 9 * 43 * 32 == 12384
    assert profsum.sweep_blocks(2, 129, 8, 0) == 3 * 32


def test_kernel_names():
    assert profsum.pass_kernel(3, 16, 2, ir=True, wv=8, pairs=1) == "mg::k_ir3d_p<16, 2, 0, 8, float>"
    assert profsum.pass_kernel(3, 16, 2, ir=True, wv=8, pairs=1, word=2) == "mg::k_ir3d_p<16, 2, 0, 8, _Float16>"
    assert profsum.pass_kernel(3, 8, 1, ir=False, wv=4, pairs=1) == "mg::k_norm3d_p<8, 1, 4>"
    assert profsum.pass_kernel(3, 16, 1, var=True, ir=True, wv=4) == "mg::k_ir3d<true, 16, 1, 0, 4>"
    assert profsum.pass_kernel(2, 16, 2, ir=True, pairs=1) == "mg::k_ir2d_p<2, 0, float>"
    assert profsum.pass_kernel(2, 16, 1, ir=False, pairs=1) == "mg::k_norm2d_p<1>"
    assert profsum.sweep_kernel(3, 4, 16, 1, wv=4) == "mg::k_smooth3d<float, 0, false, 16, 1, 0, 4>"
    assert profsum.sweep_kernel(3, 4, 8, 2, wv=1) == "mg::k_smooth3d_rc<float, 0, false, 8, 2, 0>"
    assert profsum.sweep_kernel(3, 8, 32, 1, wv=8) == "mg::k_smooth3d<double, 0, false, 32, 1, 0, 8>"
    assert profsum.sweep_kernel(3, 2, 16, 2, wv=8) == "mg::k_smooth3d<_Float16, 0, false, 16, 2, 0, 8>"
    assert profsum.sweep_kernel(3, 8, 16, 2, wv=8, flags=4) == "mg::k_smooth3d<double, 0, false, 16, 2, 4, 8>"
    assert profsum.sweep_kernel(2, 8, 32, 1, flags=4) == "mg::k_smooth2d<double, 0, false, 32, 4>"
