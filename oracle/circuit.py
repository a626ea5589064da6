"""Circuit graph, spanning tree and fundamental loops (oracle).

Paper Sec. II-D (Table I: triangle -> node, edge -> branch) and Sec. III
(tree, twigs, links, fundamental loops, Eqs. VolT / CurT / LoopVandI, voltage
sources as extra links, Eq. FinalME).

Readings fixed here (the paper leaves them open):
* each contact face (a port's source or sink triangle set) is merged into one
  equipotential node whose id is its lowest triangle index; edges inside a
  contact face become self-loop branches (always links);
* mesh edge e is the branch node(T+) -> node(T-); port k adds a
  zero-impedance source branch K_k -> S_k (sink node to source node), which
  is never a twig;
* the tree is a breadth-first forest, one root per connected component at its
  lowest node id, neighbours visited in (neighbour id, branch id) order;
* links are numbered in branch order (mesh edges, then source branches).
"""
from collections import deque
import numpy as np
import scipy.sparse as sp


class Circuit:
    def __init__(self, mesh, ports):
        n = mesh.ntri
        node = np.arange(n)
        owner = np.full(n, -1)
        sets = []
        self.port_src_node, self.port_snk_node = [], []
        for k, (src, snk) in enumerate(ports):
            ids = []
            for S in (src, snk):
                S = np.unique(np.asarray(S, dtype=np.int64))
                if S.size == 0:
                    raise ValueError("empty contact set")
                key = tuple(S.tolist())
                if key in sets:
                    sid = sets.index(key)
                else:
                    if np.any(owner[S] >= 0):
                        raise ValueError("overlapping contact sets")
                    sid = len(sets)
                    sets.append(key)
                    owner[S] = sid
                    node[S] = S.min()
                ids.append(int(min(key)))
            self.port_src_node.append(ids[0])
            self.port_snk_node.append(ids[1])
        self.node_of_tri = node
        self.contact = owner >= 0
        self.nodes = np.unique(node)
        b = mesh.nedge
        p = len(ports)
        bu = np.concatenate([node[mesh.tplus], np.array(self.port_snk_node, dtype=np.int64)])
        bv = np.concatenate([node[mesh.tminus], np.array(self.port_src_node, dtype=np.int64)])
        self.branch_u, self.branch_v = bu, bv
        self.nbranch = b + p
        self.nmesh_branch = b
        self.nport = p
        # adjacency over mesh branches that are not self-loops
        adj = {int(x): [] for x in self.nodes}
        for e in range(b):
            u, v = int(bu[e]), int(bv[e])
            if u != v:
                adj[u].append((v, e))
                adj[v].append((u, e))
        for x in adj:
            adj[x].sort()
        parent = {}
        parent_branch = {}
        depth = {}
        comp = {}
        ncomp = 0
        twig = np.zeros(b + p, dtype=bool)
        for root in self.nodes:
            root = int(root)
            if root in comp:
                continue
            comp[root] = ncomp
            parent[root] = -1
            parent_branch[root] = -1
            depth[root] = 0
            dq = deque([root])
            while dq:
                x = dq.popleft()
                for y, e in adj[x]:
                    if y not in comp:
                        comp[y] = ncomp
                        parent[y] = x
                        parent_branch[y] = e
                        depth[y] = depth[x] + 1
                        twig[e] = True
                        dq.append(y)
            ncomp += 1
        self.ncomp = ncomp
        self.comp = comp
        self.parent, self.parent_branch, self.depth = parent, parent_branch, depth
        for k in range(p):
            if comp[self.port_src_node[k]] != comp[self.port_snk_node[k]]:
                raise ValueError("port %d: source and sink in different conductors" % k)
        self.twig = twig
        self.links = np.nonzero(~twig)[0]
        self.nloop = self.links.size
        # port k's loop index
        pos = {int(e): i for i, e in enumerate(self.links)}
        self.port_loop = np.array([pos[b + k] for k in range(p)], dtype=np.int64)

    def _tree_path(self, v, u):
        """Signed twigs on the tree path v -> u (traversal direction)."""
        out = []
        a, c = v, u
        up_a, up_c = [], []
        while self.depth[a] > self.depth[c]:
            up_a.append(a)
            a = self.parent[a]
        while self.depth[c] > self.depth[a]:
            up_c.append(c)
            c = self.parent[c]
        while a != c:
            up_a.append(a)
            a = self.parent[a]
            up_c.append(c)
            c = self.parent[c]
        for x in up_a:          # traverse x -> parent(x)
            e = self.parent_branch[x]
            out.append((e, 1.0 if self.branch_u[e] == x else -1.0))
        for x in reversed(up_c):  # traverse parent(x) -> x
            e = self.parent_branch[x]
            out.append((e, 1.0 if self.branch_v[e] == x else -1.0))
        return out

    def loop_matrix(self):
        """Sparse l x (b + p) loop matrix A: the row of link u -> v is +1 on the
        link plus +-1 on each twig of the tree path v -> u (+1 where the
        twig's orientation agrees with the traversal), so A V_b sums branch
        voltage drops around the loop (Eq. VolT) and A^T I_l gives branch
        currents (Eq. CurT)."""
        rows, cols, vals = [], [], []
        for i, e in enumerate(self.links):
            u, v = int(self.branch_u[e]), int(self.branch_v[e])
            rows.append(i)
            cols.append(int(e))
            vals.append(1.0)
            if u != v:
                for t, s in self._tree_path(v, u):
                    rows.append(i)
                    cols.append(int(t))
                    vals.append(s)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.nloop, self.nbranch))

    def incidence(self):
        """Node-branch incidence N (nodes x (b + p)): +1 where the branch leaves
        the node, -1 where it enters; self-loops give zero columns."""
        idx = {int(x): i for i, x in enumerate(self.nodes)}
        rows, cols, vals = [], [], []
        for e in range(self.nbranch):
            u, v = int(self.branch_u[e]), int(self.branch_v[e])
            if u == v:
                continue
            rows += [idx[u], idx[v]]
            cols += [e, e]
            vals += [1.0, -1.0]
        return sp.csr_matrix((vals, (rows, cols)), shape=(len(self.nodes), self.nbranch))
