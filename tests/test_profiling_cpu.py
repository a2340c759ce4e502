"""The rocprofv3 summariser's cold/warm split (host logic, no GPU)."""
from paper_1511_02494_amd.profiling import FLUSH, cold_flags, cold_warm_means

F = FLUSH + "(unsigned int __vector(4)*, long)"
A = "void spmvsel::k_rowstream_slices<double, 1, false>(...)"
B = "void spmvsel::k_slice_finish<double>(...)"
T = "void at::native::vectorized_elementwise_kernel<...>"


def test_cold_flags_follow_flushes():
    seq = [A, B, A, B, F, A, B, A, B, F, A, T, F, T, A, A, F, F, A]
    assert cold_flags(seq) == [False, False, False, False, False, True, True, False, False,
                               False, True, True, False, True, True, False, False, False, True]


def test_cold_warm_means():
    seq = [(A, 10.0), (B, 1.0), (F, 99.0), (A, 20.0), (B, 3.0), (A, 12.0), (B, None)]
    m = cold_warm_means(seq)
    assert m[A]["cold_n"] == 1 and m[A]["cold_mean"] == 20.0   # the second A starts a new execute
    assert m[A]["warm_n"] == 2 and m[A]["warm_mean"] == 11.0
    assert m[B]["cold_n"] == 1 and m[B]["cold_mean"] == 3.0 and m[B]["warm_mean"] == 1.0
