"""State checkpoints on the host: State.save writes every array of a state to
one .npz file and State.load rebuilds an equal state (same optional arrays,
schedule and dense-output times), without unpickling anything.  (That a
loaded state resumes bitwise on the GPU is test_gpu_parity.py's
test_resume_from_a_checkpoint_file_is_bitwise.)"""
import numpy as np
import pytest
import torch

import paper_1706_07062_amd as K


@pytest.mark.parametrize("k_cross,constants,schedule,t_out", [(3, True, "geodesics", [1.0, 2.0, 50.0]),
                                                               (0, False, "tiles", None),
                                                               (1, True, None, None)])
def test_state_checkpoint_round_trip(tmp_path, k_cross, constants, schedule, t_out):
    st = K.State(777, k_cross=k_cross, constants=constants, device="cpu", schedule=schedule, t_out=t_out)
    g = torch.Generator().manual_seed(17)
    for name in K.State._ARRAYS:
        t = getattr(st, name)
        if t is None or name == "t_out":
            continue
        if t.dtype == torch.float64:
            t.copy_(torch.randn(t.shape, generator=g, dtype=torch.float64))
        else:
            t.copy_(torch.randint(-5, 1000, t.shape, generator=g, dtype=torch.int32))
    if st.cross is not None:
        st.cross[::7] = float("nan")
    path = tmp_path / "state.npz"
    st.save(path)
    with np.load(path, allow_pickle=False) as d:  # plain arrays only
        assert int(d["n"]) == 777 and int(d["k_cross"]) == k_cross
    st2 = K.State.load(path, device="cpu")
    assert (st2.n, st2.k_cross) == (st.n, st.k_cross)
    for name in K.State._ARRAYS:
        a, b = getattr(st, name), getattr(st2, name)
        assert (a is None) == (b is None), name
        if a is not None:
            assert a.dtype == b.dtype and a.shape == b.shape, name
            assert torch.equal(torch.nan_to_num(a, nan=-7.0) if a.is_floating_point() else a,
                               torch.nan_to_num(b, nan=-7.0) if b.is_floating_point() else b), name
    # the rebuilt descriptor points at the new arrays
    assert st2.c.n == 777 and st2.c.s == st2.s.data_ptr() and st2.c.k_cross == k_cross
