"""The sampled-column checker of the full-size GPU test, run on the CPU with
tile buffers packed from the oracle's own L and Sigma: it must report zero
error for L and rounding-level error for Sigma, and catch a planted error."""
import types

import numpy as np

from paper_2504_19171_amd import inputs
import tile_layout as lo
from paper_2504_19171_amd import stiles as st
from gpu_util import column_errors, L_TOL, SIGMA_TOL


def _tiles_from_oracle(M, f, S, b):
    lay = st.layout(M.n, M.w, M.a, b)
    w = f.w
    abL = np.zeros((w + 1, M.nb))
    for d in range(w + 1):
        abL[d, : M.nb - d] = f.Lr[d:, w - d]
    Lt = lo.host_pack(abL, f.LP, f.LC, lay)
    # Sigma's band part reaches the edge of the tile pattern, beyond w
    wide = types.SimpleNamespace(**{k: getattr(lay, k) for k in
                                    ("tile", "bt", "nt", "nb", "arrow", "arrow_ld", "off_band", "off_arrow",
                                     "off_corner", "total_doubles")})
    wide.w = S.Sb.shape[0] - 1
    St = lo.host_pack(S.Sb, S.SP, np.tril(S.SC), wide)
    return lay, Lt, St


def test_column_checker_on_oracle_tiles(oracle_mod):
    M = inputs.arrowhead_spd(700, 70, 9, seed=11)
    f = oracle_mod.cholesky(M.ab, M.P, M.C)
    S = oracle_mod.selinv(f, 64)
    lay, Lt, St = _tiles_from_oracle(M, f, S, 64)
    for j in (0, 63, 64, 333, 639, 640, 699, 700, 708):
        lerr, outside, serr, n = column_errors(Lt, St, lay, f, M, oracle_mod, j)
        assert n > 0
        assert lerr == 0.0 and outside == 0.0
        assert serr <= 1e-13
    # a planted error in one Sigma entry of column 333 is seen
    St2 = St.copy()
    band = St2[lay.off_band: lay.off_arrow].reshape(lay.nt, lay.bt + 1, 64, 64)
    J, c = divmod(333, 64)
    band[J, 1, c, 7] *= 1.0 + 1e-8
    _, _, serr, _ = column_errors(Lt, St2, lay, f, M, oracle_mod, 333)
    assert serr > SIGMA_TOL
    # and one in L
    Lt2 = Lt.copy()
    bandL = Lt2[lay.off_band: lay.off_arrow].reshape(lay.nt, lay.bt + 1, 64, 64)
    bandL[J, 0, c, c + 1] += 1e-9   # L[333 + 1][333]
    lerr, _, _, _ = column_errors(Lt2, St, lay, f, M, oracle_mod, 333)
    assert lerr > L_TOL
