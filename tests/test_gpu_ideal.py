"""Sec. 5 on the GPU: the ideal edge prolongator of a uniformly refined
triangle mesh (the coarse Whitney basis on the fine edges), given as the
initial guess with P^(n) the linear interpolation, comes out of the library's
energy minimisation unchanged when the energy is the curl-curl one (sigma
1e-12 keeps A positive definite; the mass term moves the minimiser by about
that much)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hcurl_oracle as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M", [4, 12])
def test_ideal_interpolation_survives_energy_minimisation(M):
    import paper_2506_08284_amd as P
    r = synth.refined_triangles(M)
    f = r["fine"]
    nf, nc = 2 * M + 1, M + 1
    A = synth.assemble_tri(f, np.full(f["tris"].shape[0], 1e-12), "A")
    D = O.gradient_matrix(f["tail"], f["head"], nf * nf)
    DH = O.gradient_matrix(r["coarse"]["tail"], r["coarse"]["head"], nc * nc)
    N = O.emin_pattern(D, r["Pn"], DH)[0]
    p_ideal = O.on_pattern(N, r["Pe"]).data
    Pn = r["Pn"]
    given = (Pn.indptr.astype(np.int64), Pn.indices.astype(np.int32), Pn.data.copy(), nc * nc)
    H = P.Hierarchy(A, synth.gradient_csr(f["tail"], f["head"]), [r["agg"]], n_nodes=nf * nf, nodal_prolongator=given,
                    init_guess=1, init_values=np.ascontiguousarray(p_ideal), emin_iters_given=3, record_energy=1)
    arrs, shape = H.export_csr(0, "Pe")
    Pe = sp.csr_matrix((arrs[2], arrs[1], arrs[0]), shape=shape)
    assert np.array_equal(Pe.indptr, N.indptr) and np.array_equal(Pe.indices, N.indices)
    assert abs(Pe.data - p_ideal).max() <= 1e-10 * abs(p_ideal).max()
    E = H.export_vec(0, "energy")
    assert abs(E[-1] - E[0]) <= 1e-10 * abs(E[0])
    H.close()
