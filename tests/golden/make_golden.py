"""Writes the golden fixtures in this folder. Coreness values are closed forms of the paper's
constructions or a hand derivation recorded in the fixture; nothing here runs any k-core code."""
import itertools
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def write(name, **fx):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(fx, f, indent=1)
        f.write("\n")


def grid_edges(s):
    e = []
    for i in range(s):
        for j in range(s):
            if j + 1 < s:
                e.append([i * s + j, i * s + j + 1])
            if i + 1 < s:
                e.append([i * s + j, (i + 1) * s + j])
    return e


def cube_edges(s):
    vid = lambda i, j, k: (i * s + j) * s + k
    e = []
    for i, j, k in itertools.product(range(s), repeat=3):
        if i + 1 < s: e.append([vid(i, j, k), vid(i + 1, j, k)])
        if j + 1 < s: e.append([vid(i, j, k), vid(i, j + 1, k)])
        if k + 1 < s: e.append([vid(i, j, k), vid(i, j, k + 1)])
    return e


if __name__ == "__main__":
    write("grid_5x5.json",
          citation="Sec. 6.1.1 (GRID) and Table 2: a 2D grid has k_max = 2; every vertex of a plain "
                   "s x s grid (s >= 2) lies in the 2-core and no vertex of degree <= 3 boundary "
                   "survives into a 3-core, so coreness is 2 everywhere.",
          n=25, edges=grid_edges(5), coreness=[2] * 25, kmax=2)
    write("cube_3x3x3.json",
          citation="Sec. 6.1.1 (CUBE) and Table 2: a 3D cube lattice has k_max = 3 (corners have "
                   "degree 3 and peel first at k = 3, taking the whole lattice with them).",
          n=27, edges=cube_edges(3), coreness=[3] * 27, kmax=3)
    K = 12
    e = [list(p) for p in itertools.combinations(range(K + 1), 2)]
    for i in range(1, K):
        e += [[K + i, c] for c in range(i)]
    write("hcns_k12.json",
          citation="Sec. 6.1.1 (HCNS) and Table 2: exactly one vertex of each coreness 1 <= i < "
                   "k_max plus a dense subgraph of coreness k_max. Read as a (K+1)-clique plus "
                   "u_i adjacent to i clique vertices; at K = 50000 this gives the printed "
                   "n = 0.1M and m = 5.0B. Scaled to K = 12.",
          n=2 * K, edges=e, coreness=[K] * (K + 1) + list(range(1, K)), kmax=K)
    write("worked_example_kmax3.json",
          citation="Definition of k-core and coreness (Sec. 1, Sec. 2); a worked example with "
                   "k_max = 3 in the manner of Fig. 1, derived by hand.",
          derivation="k=0 peels isolated 9. k=1 peels 8, 10, 11; 7 then has degree 1 and is "
                     "peeled, dropping 6 to 2. k=2 peels 5 and 6 (degree 2), which drops 4 to 2, "
                     "so 4 is peeled; 0 and 1 drop to 3. k=3 peels the remaining K4 {0,1,2,3}.",
          n=12,
          edges=[[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3], [4, 0], [4, 1], [4, 5], [4, 6],
                 [5, 6], [6, 7], [7, 8], [10, 11]],
          coreness=[3, 3, 3, 3, 2, 2, 2, 1, 1, 0, 1, 1], kmax=3)
