"""CPU-only checks of the HIP library: it loads, exports what include/ declares,
and its host tracker produces the same characteristics as the oracle's."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2102_01734_amd as rt
    L = rt.lib()
    names = _declared_functions()
    assert {"rt_create_grid", "rt_formal_solution", "rt_ali_step", "rt_solve"} <= names
    for n in names:
        assert hasattr(L, n), n
    assert "gfx950" in rt.rt_version()


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's sizes and offsets."""
    import subprocess
    import paper_2102_01734_amd.rt3d as b
    structs = {"rt_grid_desc": b.RtGridDesc, "rt_state": b.RtState, "rt_solve_opts": b.RtSolveOpts,
               "rt_solve_report": b.RtSolveReport}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rt3d.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.split("\n") if l)
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


@pytest.mark.parametrize("Nz,n_mu,n_phi", [(9, 4, 8), (33, 8, 16), (129, 32, 64)])
def test_library_tracker_matches_oracle_tracker(orc, Nz, n_mu, n_phi):
    """Two independent tracker formulations (DDA stepping vs sorted crossings
    located by midpoints) give identical voxel sequences and path lengths."""
    import paper_2102_01734_amd as rt
    mu, phi, _ = orc.quadrature(n_mu, n_phi)
    dirs = range(mu.size) if mu.size <= 128 else range(0, mu.size, 37)
    for d in dirs:
        a = rt.rt_box_template(Nz, n_mu, n_phi, d)
        b = orc.box_template(Nz, mu[d], phi[d])
        np.testing.assert_array_equal(a["di"], b["di"])
        np.testing.assert_array_equal(a["dj"], b["dj"])
        np.testing.assert_array_equal(a["kk"], b["kk"])
        np.testing.assert_allclose(a["s"], b["s"], rtol=0, atol=1e-13 * Nz / abs(mu[d]))


@pytest.mark.parametrize("Nr,Nt,Np,n_mu,n_phi", [(9, 8, 12, 4, 8), (6, 7, 5, 2, 4), (12, 10, 16, 8, 16)])
def test_library_sphere_tracker_matches_oracle(orc, Nr, Nt, Np, n_mu, n_phi):
    """The library's spherical tracker and the oracle's give the same
    characteristics (foot points, ranges, kinds), voxel sequences and path
    lengths; odd Nt has no equatorial plane, n_mu = 2 has no pole-near rays."""
    import paper_2102_01734_amd as rt
    g = orc.SphereGrid(Nr, Nt, Np, 1.0, 2.0)
    desc = rt.sphere_desc(Nr, Nt, Np, 1.0, 2.0, n_mu, n_phi)
    mu, phi, _ = orc.quadrature(n_mu, n_phi)
    dirs = range(mu.size) if mu.size <= 32 else range(0, mu.size, 11)
    for d in dirs:
        n = orc.direction_vector(mu[d], phi[d])
        a = rt.rt_sphere_tracks(desc, d)
        assert a["h"] == pytest.approx(g.spacing(), rel=1e-15)
        ch = g.rays(n)
        assert a["chars"].shape[0] == ch.shape[0]
        np.testing.assert_allclose(a["chars"][:, :5], ch[:, :5], rtol=0, atol=1e-14)
        np.testing.assert_array_equal(a["chars"][:, 5], ch[:, 5])
        for c in range(ch.shape[0]):
            v, s, _ = g.segments(ch[c], n)
            b0, b1 = a["begin"][c], a["begin"][c + 1]
            np.testing.assert_array_equal(a["vox"][b0:b1], v)
            np.testing.assert_allclose(a["s"][b0:b1], s, rtol=0, atol=1e-14)


def test_sphere_tracker_rejects_bad_descriptors():
    import paper_2102_01734_amd as rt
    with pytest.raises(rt.RtError):
        rt.rt_sphere_tracks(rt.sphere_desc(4, 4, 4, 2.0, 1.0, 4, 8), 0)      # r_core > r_out
    with pytest.raises(rt.RtError):
        rt.rt_sphere_tracks(rt.sphere_desc(4, 4, 4, 1.0, 2.0, 3, 8), 0)      # odd n_mu
    with pytest.raises(rt.RtError):
        rt.rt_sphere_tracks(rt.sphere_desc(4, 4, 4, 1.0, 2.0, 4, 8, source_distance=0.5), 0)
    with pytest.raises(rt.RtError):
        rt.rt_sphere_tracks(rt.sphere_desc(4, 4, 4, 1.0, 2.0, 4, 8), 32)     # direction out of range


def test_tracker_rejects_bad_requests():
    import paper_2102_01734_amd as rt
    with pytest.raises(rt.RtError):
        rt.rt_box_template(0, 4, 8, 0)
    with pytest.raises(rt.RtError):
        rt.rt_box_template(5, 3, 8, 0)       # odd n_mu would contain mu = 0
    with pytest.raises(rt.RtError):
        rt.rt_box_template(5, 4, 8, 32)      # direction out of range


def test_product_package_does_not_reference_the_oracle():
    """The GPU path must not route through the oracle: no import of it anywhere
    in the package sources or the C ABI."""
    pkg = os.path.join(ROOT, "paper_2102_01734_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if os.path.isdir(path) or path.endswith((".so", ".o", ".pyc")):
            continue
        src = open(path, errors="ignore").read()
        assert "import oracle" not in src and "from oracle" not in src and "rt_oracle" not in src, path
