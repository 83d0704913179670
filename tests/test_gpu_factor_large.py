"""Factorisation of large plane blocks, one test per kernel instance.

The sub-panel kernel picks its workgroup size, rows per thread and
sub-panel width from the largest block (513-1024, -1536, -2048, -2304,
-3072, -4096 rows), and blocks of more than 4096 rows take the generic panel
kernel.  Each case here is a 3D box split in two along z, one subdomain
across x and y, so that its planes have the stated size; the oracle would
need minutes to factor blocks of thousands of rows, so the GPU's local
solves are checked through the oracle's own subdomain operators instead:
||A_a x_a - g_a|| / ||g_a|| for every subdomain and RHS (a property that
holds at any size), and FP64 against complex64 local solves.
"""
import numpy as np
import pytest
import torch

import ddm_inputs as di
import paper_1807_04180_amd as ddm
from oracle import Oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# M cells, planes of (M + 5)^2 nodes with n_pml = 3: the instance each size selects
CASES = [
    (32, 1369),   # 512 threads, 3 rows per thread, 8-column sub-panels
    (40, 2025),   # 512 threads, 4 rows per thread
    (42, 2209),   # 768 threads, 3 rows per thread (the instance of the 3D 96^3 workload's 2116-row planes)
    (46, 2601),   # 1024 threads, 3 rows per thread, 4-column sub-panels
    (58, 3969),   # 1024 threads, 4 rows per thread
    (60, 4225),   # above 4096 rows: the generic panel kernel, one update per panel
]


@pytest.mark.parametrize("M,bs", CASES)
def test_large_plane_local_solves_by_residual(M, bs):
    w = di.small_3d(M=M, N=(1, 1, 2), n_pml=3, n_ov=2, nrhs=2, seed=7)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    for a in range(o.nsub):
        d = o.subdomain(a)
        assert (d["ext_hi"][0] - d["ext_lo"][0] + 1) * (d["ext_hi"][1] - d["ext_lo"][1] + 1) == bs
    gin = di.random_field((2, o.etot), seed=84)
    g = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), _t(w.k2.reshape(-1)), 2)
    x64 = g.local_solve(_t(gin)).cpu().numpy()
    g.close()
    for a in range(o.nsub):
        d = o.subdomain(a)
        sl = slice(d["off"], d["off"] + d["n"])
        for q in range(2):
            r = o.apply_local(a, x64[q, sl]) - gin[q, sl]
            rel = np.linalg.norm(r) / np.linalg.norm(gin[q, sl])
            assert rel < 1e-10, (a, q, rel)
    # complex64 inverses (rounded from the same FP64 factorisation) agree to
    # complex64 accuracy
    gm = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=True), _t(w.k2.reshape(-1)), 2)
    x32 = gm.local_solve(_t(gin)).cpu().numpy()
    gm.close()
    err = np.linalg.norm(x32 - x64, axis=1) / np.linalg.norm(x64, axis=1)
    assert err.max() < 5e-4, err
    torch.cuda.empty_cache()
