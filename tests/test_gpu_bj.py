"""Block-Jacobi setup (Section 4.5) on random face blocks of every size class of the inversion
kernels (one wave per face up to an edge of 64, one workgroup with the block in LDS above),
against the oracle's dense inverses, and the flagging of singular and non-finite blocks."""
import sys

import numpy as np
import pytest
import torch

from oracle import krylov

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2512_13619_amd import hdg
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return hdg.Context(0)


def face_dims(nf, ncomp, npf):
    # two faces per element (nlfe = 2): three block slots per face row
    return {"ne": 1, "nf": nf, "ncomp": ncomp, "dim": 2, "npe": 1, "npf": npf, "nlfe": 2}


def random_blocks(nf, nb, seed):
    """K[f][s][col][row] with standard normal slot-0 blocks (pivoting needed throughout) and
    random other slots (which the setup must not read)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nf, 3, nb, nb))


# (ncomp, npf): block edges 5, 16, 17, 30, 45, 48, 64 (one wave per face) and 65 (LDS)
SIZES = [(1, 5), (1, 16), (1, 17), (5, 6), (5, 9), (3, 16), (4, 16), (5, 13)]


@pytest.mark.parametrize("ncomp,npf", SIZES)
def test_bj_inverse_random_blocks(ctx, ncomp, npf):
    nb, nf = ncomp * npf, 37                 # 37 faces: the last workgroup of four is ragged
    say("bj random", nb)
    K = random_blocks(nf, nb, 100 + nb)
    B64 = torch.zeros(nf, nb, nb, dtype=torch.float64, device="cuda")
    B32 = torch.zeros(nf, nb, nb, dtype=torch.float32, device="cuda")
    ctx.bj_setup(face_dims(nf, ncomp, npf), torch.as_tensor(K).cuda().contiguous(), B64, B32)
    ref = krylov.bj_inverses(K)
    got = B64.cpu().numpy()
    for f in range(nf):
        # backward-stable inversion: error relative to the inverse, scaled by the condition number
        cond = np.linalg.cond(K[f, 0].T)
        err = np.abs(got[f] - ref[f]).max() / np.abs(ref[f]).max()
        assert err < 1e-14 * cond * nb, (f, err, cond)
        resid = np.abs(K[f, 0].T @ got[f].T - np.eye(nb)).max()
        assert resid < 1e-14 * cond * nb, (f, resid, cond)
    assert np.array_equal(B32.cpu().numpy(), got.astype(np.float32))


@pytest.mark.parametrize("ncomp,npf", [(3, 16), (5, 13)])
def test_bj_flags_singular_and_nonfinite_blocks(ctx, ncomp, npf):
    from paper_2512_13619_amd import hdg
    nb, nf = ncomp * npf, 24
    say("bj flags", nb)
    dims = face_dims(nf, ncomp, npf)
    B64 = torch.zeros(nf, nb, nb, dtype=torch.float64, device="cuda")
    K = random_blocks(nf, nb, 7)
    K[9, 0, 4, :] = 0.0                      # a zero column: singular
    with pytest.raises(hdg.HdgError, match="face 9"):
        ctx.bj_setup(dims, torch.as_tensor(K).cuda().contiguous(), B64)
    K = random_blocks(nf, nb, 8)
    K[20, 0] = 0.0                           # a zero block
    K[11, 0, 5, 3] = np.nan                  # a NaN entry: the lowest flagged face is named
    with pytest.raises(hdg.HdgError, match="face 11"):
        ctx.bj_setup(dims, torch.as_tensor(K).cuda().contiguous(), B64)
    K = random_blocks(nf, nb, 9)             # the status is cleared between calls
    ctx.bj_setup(dims, torch.as_tensor(K).cuda().contiguous(), B64)
