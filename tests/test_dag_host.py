"""Host checks of the tent dependency graph behind the persistent schedule (section 2: a
tent may be evolved once the tents it depends on are done).  The library's graph is
compared with an independent construction from the exported tent list and the mesh
cells, and, on small meshes, with the brute-force requirement: any two tents whose
patches share an element, or one of which reads the other's vertex time, are ordered by
a dependency path in the direction of their layers."""
import numpy as np
import pytest

from mtp_inputs import meshes
from paper_1906_11029_amd import mtp


def _neighbours(cells, nv):
    nb = [set() for _ in range(nv)]
    for c in np.asarray(cells):
        for a in c:
            nb[a].update(int(b) for b in c if b != a)
    return nb


def _preds_independent(vertex, layer, nb):
    """Predecessors from per-vertex tent lists: for tent i at V, the tent at u in {V} and
    the neighbours of V with the largest layer below layer[i]."""
    per_vertex = {}
    for i, v in enumerate(vertex):
        per_vertex.setdefault(int(v), []).append(i)
    preds = []
    for i, v in enumerate(vertex):
        p = set()
        for u in {int(v)} | nb[int(v)]:
            cand = [j for j in per_vertex.get(u, []) if layer[j] < layer[i]]
            if cand:
                p.add(max(cand, key=lambda j: layer[j]))
        preds.append(p)
    return preds


def _library_preds(dag, n):
    preds = [set() for _ in range(n)]
    sp, sc = dag["succ_ptr"], dag["succ"]
    for i in range(n):
        for k in range(sp[i], sp[i + 1]):
            preds[int(sc[k])].add(i)
    return preds


CASES = [("2d", 4, 0.5), ("2d", 8, 0.5), ("3d", 2, 0.4), ("3d", 3, 0.3), ("graded", 3, 0.2),
         ("disk_colour", 4, 0.2), ("3d_colour", 2, 0.3)]


def _setup(kind, n, T):
    if kind == "disk_colour":       # tables of the colour rule
        mm = meshes.disk_tri(n)
        M = mtp.Mesh(mm["coords"], mm["cells"])
        return mm, M, mtp.Tents(M, T, 0.5, rule=mtp.MTP_PITCH_COLOUR)
    if kind == "3d_colour":
        mm = meshes.cube_kuhn(n)
        M = mtp.Mesh(mm["coords"], mm["cells"])
        return mm, M, mtp.Tents(M, T, 0.5, rule=mtp.MTP_PITCH_COLOUR)
    if kind == "2d":
        mm = meshes.square_tri(n)
        M = mtp.Mesh(mm["coords"], mm["cells"])
    elif kind == "3d":
        mm = meshes.cube_kuhn(n)
        M = mtp.Mesh(mm["coords"], mm["cells"])
    else:
        mm = meshes.cube_kuhn(n, axis_map=lambda g: 0.3 * g + 0.7 * g * g)
        eps, mu = meshes.materials_split(mm)
        M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu)
    return mm, M, mtp.Tents(M, T, 0.5)


@pytest.mark.parametrize("kind,n,T", CASES)
def test_dag_matches_independent_construction(kind, n, T):
    mm, M, tents = _setup(kind, n, T)
    ex = tents.export()
    dag = tents.dag()
    nt = tents.n_tents
    nb = _neighbours(mm["cells"], M.info["nv"])
    want = _preds_independent(ex["vertex"], ex["layer"], nb)
    got = _library_preds(dag, nt)
    assert got == want
    assert np.array_equal(dag["pred_count"], [len(p) for p in want])
    # the tents without dependency are exactly the first layer, a prefix of the table
    assert dag["n_ready"] == tents.layer_ptr[1]
    assert (dag["pred_count"][:dag["n_ready"]] == 0).all() and (dag["pred_count"][dag["n_ready"]:] > 0).all()
    # successor lists are sorted in table order and point forward
    sp, sc = dag["succ_ptr"], dag["succ"]
    for i in range(nt):
        s = sc[sp[i]:sp[i + 1]]
        assert (np.diff(s) > 0).all() and (s > i).all()


@pytest.mark.parametrize("kind,n,T", CASES[:3] + [("graded", 2, 0.2), ("disk_colour", 3, 0.2)])
def test_dag_orders_every_conflicting_pair(kind, n, T):
    mm, M, tents = _setup(kind, n, T)
    ex = tents.export()
    dag = tents.dag()
    nt = tents.n_tents
    assert nt <= 1500
    nb = _neighbours(mm["cells"], M.info["nv"])
    # reachability by repeated boolean products (tents are in a topological order)
    R = np.zeros((nt, nt), dtype=bool)
    sp, sc = dag["succ_ptr"], dag["succ"]
    for i in range(nt - 1, -1, -1):
        for k in range(sp[i], sp[i + 1]):
            j = int(sc[k])
            R[i, j] = True
            R[i] |= R[j]
    v, lay = ex["vertex"], ex["layer"]
    for i in range(nt):
        for j in range(i + 1, nt):
            if int(v[j]) == int(v[i]) or int(v[j]) in nb[int(v[i])]:
                assert lay[i] != lay[j]
                a, b = (i, j) if lay[i] < lay[j] else (j, i)
                assert R[a, b] and not R[b, a], (i, j)
