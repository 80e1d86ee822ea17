"""Exact rational reference for the advection part of the step (test helper).

Given rational vertices, vertex/face velocities, dt and *unnormalised*
rational PLIC planes, every quantity of the advection step is a rational
function of the inputs: face area vectors, V_d, the FMFPA lateral-plane
normals, line directions and back-vertex projections, the EMFPA streak-line
back vertices and lateral-face centres, the NMFPA translated faces, the apex
shift, every clip point and
every volume.  This module recomputes them with Python
Fractions, so its answers carry no rounding error at all.

It is written independently of the oracle: volumes of intersections are done
by exact tetrahedron splitting (a tetrahedron cut by a plane is kept whole,
dropped, or split into one or three tetrahedra), not by face-list clipping.
It pins the oracle; it never touches the HIP library.
"""
from __future__ import annotations

from fractions import Fraction as Q

ZERO = Q(0)


def sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def scl(s, a):
    return (s * a[0], s * a[1], s * a[2])


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def det(a, b, c):
    return dot(a, cross(b, c))


def tet_signed6(t):
    return det(sub(t[1], t[0]), sub(t[2], t[0]), sub(t[3], t[0]))


def _lerp(p, sp, q, sq):
    # point where the linear function s is zero on segment p-q (sp, sq of opposite sign)
    t = sp / (sp - sq)
    return add(p, scl(t, sub(q, p)))


def split_keep(tet, n, d):
    """Tetrahedra covering tet ∩ {n.x + d >= 0} (exact)."""
    s = [dot(n, p) + d for p in tet]
    pos = [i for i in range(4) if s[i] > 0]
    neg = [i for i in range(4) if s[i] < 0]
    if not neg:
        return [tet]
    if not pos:
        return []
    zer = [i for i in range(4) if s[i] == 0]
    # treat on-plane vertices as kept
    keep = pos + zer
    drop = neg
    P = tet
    if len(keep) == 1:
        a = keep[0]
        return [(P[a],) + tuple(_lerp(P[a], s[a], P[b], s[b]) for b in drop)]
    if len(keep) == 3:
        d0 = drop[0]
        a, b, c = keep
        pa = _lerp(P[a], s[a], P[d0], s[d0]) if s[a] != 0 else P[a]
        pb = _lerp(P[b], s[b], P[d0], s[d0]) if s[b] != 0 else P[b]
        pc = _lerp(P[c], s[c], P[d0], s[d0]) if s[c] != 0 else P[c]
        # prism (a,b,c | pa,pb,pc)
        return [(P[a], P[b], P[c], pa), (P[b], P[c], pa, pb), (P[c], pa, pb, pc)]
    # two kept (a, b), two dropped (c, d)
    a, b = keep
    c, d_ = drop
    p1 = _lerp(P[a], s[a], P[c], s[c]) if s[a] != 0 else P[a]
    p2 = _lerp(P[a], s[a], P[d_], s[d_]) if s[a] != 0 else P[a]
    p3 = _lerp(P[b], s[b], P[c], s[c]) if s[b] != 0 else P[b]
    p4 = _lerp(P[b], s[b], P[d_], s[d_]) if s[b] != 0 else P[b]
    # wedge with end triangles (a, p1, p2) and (b, p3, p4)
    return [(P[a], p1, p2, P[b]), (p1, p2, P[b], p4), (p1, P[b], p4, p3)]


def clip_volume(tet, planes):
    """Exact vol(tet ∩ {n.x + d >= 0 for all (n, d)})."""
    tets = [tet]
    for (n, d) in planes:
        nxt = []
        for t in tets:
            nxt.extend(split_keep(t, n, d))
        tets = nxt
        if not tets:
            return ZERO
    return sum(abs(tet_signed6(t)) for t in tets) / 6


def tet_inward_planes(t):
    a, b, c, d = t
    if tet_signed6(t) < 0:
        c, d = d, c
    out = []
    for (p, q, r) in ((a, c, b), (a, b, d), (a, d, c), (b, c, d)):
        N = cross(sub(q, p), sub(r, p))
        out.append(((-N[0], -N[1], -N[2]), dot(N, p)))
    return out


def box_planes(lo, hi):
    return [((Q(1), ZERO, ZERO), -lo[0]), ((Q(-1), ZERO, ZERO), hi[0]),
            ((ZERO, Q(1), ZERO), -lo[1]), ((ZERO, Q(-1), ZERO), hi[1]),
            ((ZERO, ZERO, Q(1)), -lo[2]), ((ZERO, ZERO, Q(-1)), hi[2])]


class ExactMesh:
    def __init__(self, verts, fv_ptr, fv_idx, owner, neigh, nc):
        self.X = [tuple(Q(c) for c in v) for v in verts]
        self.nv = len(self.X)
        self.faces = [list(fv_idx[fv_ptr[f]:fv_ptr[f + 1]]) for f in range(len(owner))]
        self.owner = list(owner)
        self.neigh = list(neigh)
        self.nf = len(owner)
        self.nc = nc
        self.cf = [[] for _ in range(nc)]
        for f in range(self.nf):
            self.cf[self.owner[f]].append((f, 1))
            if self.neigh[f] >= 0:
                self.cf[self.neigh[f]].append((f, -1))
        self.cv = []
        for c in range(nc):
            vs = sorted({v for (f, _) in self.cf[c] for v in self.faces[f]})
            self.cv.append(vs)
        vc = [[] for _ in range(self.nv)]
        for c in range(nc):
            for v in self.cv[c]:
                vc[v].append(c)
        self.nb = []
        for c in range(nc):
            self.nb.append(sorted({k for v in self.cv[c] for k in vc[v] if k != c}))
        # geometry
        self.fc, self.S = [], []
        for f in range(self.nf):
            pts = [self.X[v] for v in self.faces[f]]
            k = len(pts)
            c = (sum(p[0] for p in pts) / k, sum(p[1] for p in pts) / k, sum(p[2] for p in pts) / k)
            A = (ZERO, ZERO, ZERO)
            for i in range(k):
                A = add(A, cross(sub(pts[i], c), sub(pts[(i + 1) % k], c)))
            self.fc.append(c)
            self.S.append(scl(Q(1, 2), A))
        self.cc, self.lo, self.hi, self.isbox, self.tets, self.V = [], [], [], [], [], []
        for c in range(nc):
            pts = [self.X[v] for v in self.cv[c]]
            k = len(pts)
            cen = (sum(p[0] for p in pts) / k, sum(p[1] for p in pts) / k, sum(p[2] for p in pts) / k)
            lo = tuple(min(p[a] for p in pts) for a in range(3))
            hi = tuple(max(p[a] for p in pts) for a in range(3))
            box = (k == 8 and len(self.cf[c]) == 6 and all(len(self.faces[f]) == 4 for f, _ in self.cf[c])
                   and all(p[a] in (lo[a], hi[a]) for p in pts for a in range(3))
                   and len({tuple(p[a] == hi[a] for a in range(3)) for p in pts}) == 8)
            tris = []
            for (f, sg) in self.cf[c]:
                vs = [self.X[v] for v in self.faces[f]]
                if len(vs) == 3:
                    tris.append(tuple(vs) if sg > 0 else (vs[0], vs[2], vs[1]))
                else:
                    for i in range(len(vs)):
                        a, b = vs[i], vs[(i + 1) % len(vs)]
                        tris.append((self.fc[f], a, b) if sg > 0 else (self.fc[f], b, a))
            tets = [(cen,) + t for t in tris]
            vol = sum(det(sub(t[1], cen), sub(t[2], cen), sub(t[3], cen)) for t in tets) / 6
            self.cc.append(cen); self.lo.append(lo); self.hi.append(hi); self.isbox.append(box)
            self.tets.append(tets); self.V.append(vol)

    def candidates(self, f):
        o, n = self.owner[f], self.neigh[f]
        s = {o} | set(self.nb[o])
        if n >= 0:
            s |= {n} | set(self.nb[n])
        return sorted(s)

    def tet_cell_volume(self, T, c, plane):
        extra = [plane] if plane is not None else []
        if self.isbox[c]:
            return clip_volume(T, box_planes(self.lo[c], self.hi[c]) + extra)
        acc = ZERO
        for s in self.tets[c]:
            d6 = tet_signed6(s)
            if d6 == 0:
                continue
            v = clip_volume(T, tet_inward_planes(s) + extra)
            acc += v if d6 > 0 else -v
        return acc

    def fmfpa(self, f, u_vert, dt, Vd, degen=Q(1, 10 ** 12)):
        """Exact FMFPA polyhedron: returns (tets with signs, x, b, apex, degenerate)."""
        vs = self.faces[f]
        I = len(vs)
        x = [self.X[v] for v in vs]
        u = [u_vert[v] for v in vs]
        m = []
        for i in range(I):
            j = (i + 1) % I
            ub = tuple(Q(1, 2) * (u[i][a] + u[j][a]) for a in range(3))
            m.append(cross(sub(x[j], x[i]), ub))
        b = []
        for i in range(I):
            m0, m1 = m[(i - 1) % I], m[i]
            d = cross(m0, m1)
            dd, a0, a1 = dot(d, d), dot(m0, m0), dot(m1, m1)
            if a0 == 0 or a1 == 0 or dd <= degen * a0 * a1:
                b.append(sub(x[i], scl(dt, u[i])))
            else:
                b.append(sub(x[i], scl(dt * dot(u[i], d) / dd, d)))
        g = (sum(p[0] for p in b) / I, sum(p[1] for p in b) / I, sum(p[2] for p in b) / I)
        c = self.fc[f]
        S = self.S[f]
        V0 = ZERO
        W = ZERO
        for i in range(I):
            j = (i + 1) % I
            V0 += det(sub(x[j], c), sub(x[i], c), sub(b[j], c))
            V0 += det(sub(x[i], c), sub(b[i], c), sub(b[j], c))
            V0 += det(sub(g, c), sub(b[j], c), sub(b[i], c))
            W += det(S, sub(b[j], c), sub(b[i], c))
        V0 /= 6
        W /= 6
        degenerate = abs(W) <= Q(1, 10 ** 12) * dot(S, S)
        mu = ZERO if degenerate else (Vd - V0) / W
        apex = add(g, scl(mu, S))
        tets = []
        for i in range(I):
            j = (i + 1) % I
            for t in ((c, x[j], x[i], b[j]), (c, x[i], b[i], b[j]), (c, apex, b[j], b[i])):
                d6 = tet_signed6(t)
                if d6 != 0:
                    tets.append((t, 1 if d6 > 0 else -1))
        return tets, x, b, apex, degenerate

    def emfpa(self, f, u_vert, dt, Vd):
        """Exact EMFPA polyhedron (Sec. "Edge-matched flux polyhedron").

        Returns (tets with signs, x, b, lateral centres, apex, degenerate).
        The polyhedron is described by its closed surface: the cell face, four
        triangles per lateral face about the face's vertex mean, and the back
        face fanned about the apex; its tets join each surface triangle to the
        face centre.
        """
        vs = self.faces[f]
        I = len(vs)
        x = [self.X[v] for v in vs]
        b = [sub(x[i], scl(dt, u_vert[v])) for i, v in enumerate(vs)]
        cen = []
        tris = []  # lateral triangles, outward with the back face as (apex, b_j, b_i)
        for i in range(I):
            j = (i + 1) % I
            quad = [x[j], x[i], b[i], b[j]]
            m = tuple(sum(p[a] for p in quad) / 4 for a in range(3))
            cen.append(m)
            for k in range(4):
                tris.append((quad[k], quad[(k + 1) % 4], m))
        g = tuple(sum(p[a] for p in b) / I for a in range(3))
        c = self.fc[f]
        S = self.S[f]

        def vol6(apex):
            tot = sum(det(sub(p, c), sub(q, c), sub(r, c)) for p, q, r in tris)
            for i in range(I):
                j = (i + 1) % I
                tot += det(sub(apex, c), sub(b[j], c), sub(b[i], c))
            return tot

        # the volume is affine in the apex shift along S: solve V(g + mu S) = Vd
        v0 = vol6(g) / 6
        w = vol6(add(g, S)) / 6 - v0
        degenerate = abs(w) <= Q(1, 10 ** 12) * dot(S, S)
        mu = ZERO if degenerate else (Vd - v0) / w
        apex = add(g, scl(mu, S))
        back = [(apex, b[(i + 1) % I], b[i]) for i in range(I)]
        tets = []
        for (p, q, r) in tris + back:
            t = (c, p, q, r)
            d6 = tet_signed6(t)
            if d6 != 0:
                tets.append((t, 1 if d6 > 0 else -1))
        return tets, x, b, cen, apex, degenerate

    def nmfpa(self, f, uf, dt):
        """Exact NMFPA polyhedron (Sec. "Non-matched flux polyhedron"): the face
        translated back by dt uf; its lateral faces and back face are planar, so
        any triangulation bounds the same prism.  Here the lateral
        parallelograms are split along (x_i, b_{i+1}) and the back face is
        fanned from its vertex mean; tets join each surface triangle to the face
        centre.  Returns (tets with signs, x, b)."""
        vs = self.faces[f]
        I = len(vs)
        x = [self.X[v] for v in vs]
        b = [sub(p, scl(dt, uf)) for p in x]
        g = tuple(sum(p[a] for p in b) / I for a in range(3))
        c = self.fc[f]
        tris = []
        for i in range(I):
            j = (i + 1) % I
            tris += [(x[j], x[i], b[i]), (x[j], b[i], b[j]), (g, b[j], b[i])]
        tets = []
        for (p, q, r) in tris:
            t = (c, p, q, r)
            d6 = tet_signed6(t)
            if d6 != 0:
                tets.append((t, 1 if d6 > 0 else -1))
        return tets, x, b

    def face_flux(self, f, planes, tcell, tface, u_face, u_vert, dt, method="fmfpa"):
        """Exact (Vd, VF, upwind) of face f; planes[c] = ((nx,ny,nz), C) rational."""
        Vd = dt * dot(u_face[f], self.S[f])
        up = self.owner[f] if Vd >= 0 else self.neigh[f]
        if self.neigh[f] < 0 and Vd < 0:
            return Vd, ZERO, up
        if tface[f] == -1:
            return Vd, ZERO, up
        if tface[f] == 1:
            return Vd, Vd, up
        if method == "emfpa":
            tets, *_ = self.emfpa(f, u_vert, dt, Vd)
        elif method == "nmfpa":
            tets, *_ = self.nmfpa(f, u_face[f], dt)
        else:
            tets, *_ = self.fmfpa(f, u_vert, dt, Vd)
        acc = ZERO
        cands = self.candidates(f)
        for (T, sg) in tets:
            part = ZERO
            for k in cands:
                if tcell[k] == -1:
                    continue
                pl = planes[k] if tcell[k] == 0 else None
                part += self.tet_cell_volume(T, k, pl)
            acc += part if sg > 0 else -part
        return Vd, acc, up

    def update(self, c, Vd, VF, Fin):
        VdT = sum((Vd[f] if sg > 0 else -Vd[f]) for f, sg in self.cf[c])
        VFT = sum((VF[f] if sg > 0 else -VF[f]) for f, sg in self.cf[c])
        V = self.V[c]
        h = VdT / (2 * V)
        Fn = (Fin * (1 + h) - VFT / V) / (1 - h)
        return min(max(Fn, ZERO), Q(1))
