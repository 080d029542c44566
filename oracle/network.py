"""The implicit operators on which einsumsvd runs (Sec. III-B, Alg. 3; Sec. IV-A).

Zip-up step (two-layer, Fig. 5 / Alg. 3):  the carry V[a,x,X,b,h,H] from the
previous column, the boundary tensor S[b,u,U,c] of this column, the ket site
T[u,y,h,g,p] and the bra site B[U,Y,H,G,p] (used complex-conjugated) form

    A[(a,x,X), (y,Y,c,g,G)] = sum_{b,h,H,u,U,p} V S T conj(B)

Rows are the legs that stay with the finished boundary tensor, columns the
legs that move on with the next carry.  The two layers are never merged into
one double-layer tensor (Sec. III-B, two-layer BMPS).

Pair network: two adjacent boundary tensors Bl[a,u,U,b], Br[b,v,V,c] and two
horizontally adjacent ket/bra site pairs T1[u,x,1,h,p], T2[v,y,h,1,q]:

    A[(a,x,X), (y,Y,c)] = sum Bl Br T1 conj(T1) T2 conj(T2)
"""
import numpy as np


class ImplicitOperator:
    """A linear operator known only through contractions (Alg. 4 needs A X and A^* Y)."""

    def __init__(self, rows_shape, cols_shape, fwd, adj, explicit):
        self.rows_shape = tuple(rows_shape)
        self.cols_shape = tuple(cols_shape)
        self.n_rows = int(np.prod(rows_shape))
        self.n_cols = int(np.prod(cols_shape))
        self._fwd, self._adj, self._explicit = fwd, adj, explicit

    def apply(self, X):
        k = X.shape[1]
        return self._fwd(X.reshape(self.cols_shape + (k,))).reshape(self.n_rows, k)

    def apply_adj(self, Y):
        k = Y.shape[1]
        return self._adj(Y.reshape(self.rows_shape + (k,))).reshape(self.n_cols, k)

    def explicit(self):
        return self._explicit().reshape(self.n_rows, self.n_cols)


def zipup_operator(V, S, T, B):
    a, x, X, b, h, H = V.shape
    _, u, U, c = S.shape
    _, y, _, g, _ = T.shape
    _, Y, _, G, _ = B.shape
    Bc = B.conj()

    # one pairwise contraction per tensor of the network, in the order of the
    # stages (multi-operand einsum path searches can pick orders that are
    # orders of magnitude slower); each pairwise contraction is one matrix
    # product (BLAS), the library primitive a step may use
    def fwd(Om):
        W = np.einsum("uyhgp,yYcgGj->uhpYcGj", T, Om, optimize=True)
        W = np.einsum("UYHGp,uhpYcGj->uhUHcj", Bc, W, optimize=True)
        W = np.einsum("buUc,uhUHcj->bhHj", S, W, optimize=True)
        return np.einsum("axXbhH,bhHj->axXj", V, W, optimize=True)

    def adj(P):
        W = np.einsum("axXbhH,axXj->bhHj", V.conj(), P, optimize=True)
        W = np.einsum("buUc,bhHj->uhUHcj", S.conj(), W, optimize=True)
        W = np.einsum("UYHGp,uhUHcj->uhpYcGj", B, W, optimize=True)
        return np.einsum("uyhgp,uhpYcGj->yYcgGj", T.conj(), W, optimize=True)

    def explicit():
        return np.einsum("axXbhH,buUc,uyhgp,UYHGp->axXyYcgG", V, S, T, Bc, optimize=True)

    return ImplicitOperator((a, x, X), (y, Y, c, g, G), fwd, adj, explicit)


def pair_operator(Bl, Br, T1, T2, T1b=None, T2b=None):
    T1b = T1 if T1b is None else T1b
    T2b = T2 if T2b is None else T2b
    a, u, U, b = Bl.shape
    _, v, V, c = Br.shape
    x, X, y, Y = T1.shape[1], T1b.shape[1], T2.shape[1], T2b.shape[1]
    # drop the dim-1 outer horizontal legs
    t1, t1b = T1[:, :, 0, :, :], T1b[:, :, 0, :, :].conj()
    t2, t2b = T2[:, :, :, 0, :], T2b[:, :, :, 0, :].conj()
    sub = "auUb,bvVc,uxhp,UXHp,vyhq,VYHq"

    def fwd(Om):
        W = np.einsum("vyhq,yYcj->vhqYcj", t2, Om, optimize=True)
        W = np.einsum("VYHq,vhqYcj->vhVHcj", t2b, W, optimize=True)
        W = np.einsum("bvVc,vhVHcj->bhHj", Br, W, optimize=True)
        W = np.einsum("auUb,bhHj->auUhHj", Bl, W, optimize=True)
        W = np.einsum("uxhp,auUhHj->axpUHj", t1, W, optimize=True)
        return np.einsum("UXHp,axpUHj->axXj", t1b, W, optimize=True)

    def adj(P):
        W = np.einsum("UXHp,axXj->axpUHj", t1b.conj(), P, optimize=True)
        W = np.einsum("uxhp,axpUHj->auUhHj", t1.conj(), W, optimize=True)
        W = np.einsum("auUb,auUhHj->bhHj", Bl.conj(), W, optimize=True)
        W = np.einsum("bvVc,bhHj->vhVHcj", Br.conj(), W, optimize=True)
        W = np.einsum("VYHq,vhVHcj->vhqYcj", t2b.conj(), W, optimize=True)
        return np.einsum("vyhq,vhqYcj->yYcj", t2.conj(), W, optimize=True)

    def explicit():
        return np.einsum(sub + "->axXyYc", Bl, Br, t1, t1b, t2, t2b, optimize=True)

    return ImplicitOperator((a, x, X), (y, Y, c), fwd, adj, explicit)

