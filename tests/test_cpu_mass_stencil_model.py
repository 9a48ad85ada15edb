"""Host-side model of the mass kernel's decomposition (the Kronecker-stencil
mass action): the block tiling (64 x slots per block, one element's rows of y
per wave, chunks of element layers along z), the input planes with their x
and y halos, the x-pass items, the y-pass rows and the z march with the
chunk's leading element and the vertex carry are transcribed index by index
from the kernel, for P = 1..8 in both precisions and several launch shapes,
with Dirichlet masks.  Checked: every LDS and global index stays inside its
array, every output slot is written exactly once, and the result equals the
definition -- rho detJ times the Kronecker product of the three assembled 1D
masses (each the sum over elements of the element matrix Mq placed at the
element's slots) -- applied to the masked input.  Mq is an arbitrary
symmetric positive matrix here: the model checks the decomposition, not the
1D mass of a rule (the GPU parity tests compare the kernel with the oracle)."""
import numpy as np
import pytest

NT_WAVE = 64


def dims(P, word):
    n = P + 1
    waves = (12 if P <= 5 else 8) if word == 4 else (12 if P <= 4 else 4)
    EX = 64 // P
    TX = EX * P
    RY = 4 if P == 8 else P
    GPE = P // RY
    EY = waves // GPE
    TY = EY * P
    IX, IY = TX + P + 1, TY + P + 1
    VW = 16 // word
    IXP = (IX + VW - 1) // VW * VW
    TXP = (TX + VW - 1) // VW * VW
    NT = NT_WAVE * waves
    return dict(n=n, waves=waves, NT=NT, EX=EX, TX=TX, RY=RY, GPE=GPE, EY=EY, TY=TY, IX=IX,
                IY=IY, IXP=IXP, TXP=TXP, NLD=(IX * IY + NT - 1) // NT,
                NXI=(EX * IY + NT - 1) // NT)


def grid(D, nx, ny, nz, target):
    nxt = (nx + D["EX"]) // D["EX"]
    nyt = (ny + D["EY"]) // D["EY"]
    base = nxt * nyt * 3
    nzc = min(max(target // base, 1), nz)
    cz = (nz + nzc - 1) // nzc
    nzc = (nz + cz - 1) // cz
    return nxt, nyt, nzc, cz


def xcd_order(G):
    """Logical block of each launched block (blocks b, b + 8, ... on one XCD
    take a contiguous range)."""
    per, rem = G // 8, G % 8
    out = []
    for b in range(G):
        x, k = b % 8, b // 8
        out.append(x * (per + 1) + k if x < rem else rem * (per + 1) + (x - rem) * per + k)
    return out


def run_model(P, word, n_el, Mq, v, bits, rs, target):
    nx, ny, nz = n_el
    D = dims(P, word)
    n, NT, EX, TX, RY, GPE, EY, TY = (D[k] for k in "n NT EX TX RY GPE EY TY".split())
    IX, IY, IXP, TXP, NLD, NXI = (D[k] for k in "IX IY IXP TXP NLD NXI".split())
    Nx, Ny, Nz = nx * P + 1, ny * P + 1, nz * P + 1
    Nn = Nx * Ny * Nz
    nxt, nyt, nzc, cz = grid(D, nx, ny, nz, target)
    G = nxt * nyt * nzc * 3
    order = xcd_order(G)
    assert sorted(order) == list(range(G))
    y = np.full(3 * Nn, np.nan)
    writes = np.zeros(3 * Nn, dtype=int)
    tid = np.arange(NT)
    lane, wv = tid % 64, tid // 64
    for blk in order:
        b = blk
        xt = b % nxt
        b //= nxt
        yt = b % nyt
        b //= nyt
        zc, comp = b % nzc, b // nzc
        ex0, ey0 = xt * EX, yt * EY
        ez_lo = zc * cz
        ez_hi = min(nz, ez_lo + cz)
        x0, y0 = ex0 * P, ey0 * P
        mb = bits >> comp
        # input-plane slots of the threads
        idx = tid[:, None] + NT * np.arange(NLD)[None, :]
        r, c = idx // IX, idx % IX
        gx, gy = x0 - P + c, y0 - P + r
        inplane = idx < IX * IY
        ok = (inplane & (gx >= 0) & (gx < Nx) & (gy >= 0) & (gy < Ny)
              & ~((mb & 1 > 0) & (gx == 0)) & ~((mb & 8 > 0) & (gx == Nx - 1))
              & ~((mb & 64 > 0) & (gy == 0)) & ~((mb & 512 > 0) & (gy == Ny - 1)))
        lpos = np.where(inplane, r * IXP + c, -1)
        assert lpos.max() < IY * IXP
        # x-pass items: consecutive lanes take consecutive elements of a row
        it = tid[:, None] + NT * np.arange(NXI)[None, :]
        xr, je = it // EX, it % EX
        e = ex0 + je
        act = (it < EX * IY) & (e <= nx)
        xin, xout = xr * IXP + je * P, xr * TXP + je * P
        assert (xin[act] + 2 * P).max(initial=0) < IY * IXP
        assert (xout[act] + P - 1).max(initial=0) < IY * TXP
        own, left = act & (e < nx), act & (e > 0)
        # y-pass rows of the waves
        gq, l0 = wv // GPE, (wv % GPE) * RY
        ey = ey0 + gq
        gxo = x0 + lane
        xcl = np.minimum(lane, TX - 1)
        xok = (lane < TX) & (gxo < Nx)
        assert ((gq * P + 2 * P) * TXP + xcl).max() < IY * TXP

        def plane(z):
            """The kernel's load, x pass and y pass for plane z: w[thread, j]."""
            assert 0 <= z < Nz
            zok = not ((mb & 4096 and z == 0) or (mb & 32768 and z == Nz - 1))
            sIn = np.full(IY * IXP, np.nan)
            vals = np.where(ok & zok, v[comp * Nn + z * Nx * Ny + np.where(ok, gy * Nx + gx, 0)],
                            0.0)
            sIn[lpos[inplane]] = vals[inplane]
            sX = np.full(IY * TXP, np.nan)
            a_act = act.ravel()
            xi, xo = xin.ravel()[a_act], xout.ravel()[a_act]
            ow, lf = own.ravel()[a_act], left.ravel()[a_act]
            U = sIn[xi[:, None] + np.arange(2 * P + 1)[None, :]]
            o = np.where(ow[:, None], U[:, P:] @ Mq[:P, :].T, 0.0)
            o[:, 0] += np.where(lf, U[:, :P + 1] @ Mq[P, :], 0.0)
            sX[xo] = o[:, 0]
            for l in range(1, P):
                sX[xo[ow] + l] = o[ow, l]
            colv = sX[(gq * P * TXP + xcl)[:, None] + TXP * np.arange(2 * P + 1)[None, :]]
            rows = Mq[l0[:, None] + np.arange(RY)[None, :]]  # [thread, j, a]
            w = np.where((ey < ny)[:, None], np.einsum("tja,ta->tj", rows, colv[:, P:]), 0.0)
            lt = (l0 == 0) & (ey > 0) & (ey <= ny)
            w[:, 0] += np.where(lt, colv[:, :P + 1] @ Mq[P, :], 0.0)
            return w

        orow = np.full((NT, RY), -1)
        ocon = np.zeros((NT, RY), dtype=bool)
        for j in range(RY):
            gyo = y0 + gq * P + l0 + j
            okj = xok & (gyo < Ny) & (ey <= ny)
            orow[:, j] = np.where(okj, gyo * Nx + gxo, -1)
            ocon[:, j] = (((mb & 1 > 0) & (gxo == 0)) | ((mb & 8 > 0) & (gxo == Nx - 1))
                          | ((mb & 64 > 0) & (gyo == 0)) | ((mb & 512 > 0) & (gyo == Ny - 1)))

        def emit(zo, j, val):
            sel = orow[:, j] >= 0
            con = ocon[:, j] | bool((mb & 4096 and zo == 0) or (mb & 32768 and zo == Nz - 1))
            gi = comp * Nn + zo * Nx * Ny + orow[sel, j]
            assert gi.min(initial=0) >= 0 and gi.max(initial=0) < 3 * Nn
            y[gi] = np.where(con[sel], 0.0, val[sel] * rs)
            writes[gi] += 1

        e_start = ez_lo - 1 if ez_lo > 0 else 0
        z0, zlast = e_start * P, ez_hi * P
        acc = np.zeros((NT, RY, n))
        carry = np.zeros((NT, RY))
        for z in range(z0, zlast + 1):
            w = plane(z)
            a = z % P
            if a != 0:
                acc += Mq[None, None, :, a] * w[:, :, None]
            else:
                if z > z0:
                    acc += Mq[None, None, :, P] * w[:, :, None]
                    e_done = z // P - 1
                    if e_done >= ez_lo:
                        for l in range(P):
                            for j in range(RY):
                                emit(e_done * P + l, j, acc[:, j, l])
                carry = acc[:, :, P].copy() if z > z0 else np.zeros((NT, RY))
                acc = Mq[None, None, :, 0] * w[:, :, None]
                acc[:, :, 0] += carry
        if ez_hi == nz:
            for j in range(RY):
                emit(Nz - 1, j, carry[:, j])
    return y, writes


def reference(P, n_el, Mq, v, bits, rs):
    def assembled(ne):
        A = np.zeros((ne * P + 1, ne * P + 1))
        for e in range(ne):
            A[e * P:e * P + P + 1, e * P:e * P + P + 1] += Mq
        return A
    nx, ny, nz = n_el
    Ax, Ay, Az = assembled(nx), assembled(ny), assembled(nz)
    Nn = Ax.shape[0] * Ay.shape[0] * Az.shape[0]
    out = np.zeros(3 * Nn)
    for comp in range(3):
        mb = bits >> comp
        V = v[comp * Nn:(comp + 1) * Nn].reshape(Az.shape[0], Ay.shape[0], Ax.shape[0]).copy()
        con = np.zeros(V.shape, dtype=bool)
        for bit, sl in ((1, (slice(None), slice(None), 0)), (8, (slice(None), slice(None), -1)),
                        (64, (slice(None), 0, slice(None))), (512, (slice(None), -1, slice(None))),
                        (4096, (0, slice(None), slice(None))), (32768, (-1, slice(None), slice(None)))):
            if mb & bit:
                con[sl] = True
        V[con] = 0.0
        # the Kronecker product applied one direction at a time
        Y = np.einsum("kc,cji->kji", Az, np.einsum("jb,zbi->zji", Ay, V @ Ax.T)) * rs
        Y[con] = 0.0
        out[comp * Nn:(comp + 1) * Nn] = Y.ravel()
    return out


# (P, word, mesh, Dirichlet bits, target blocks): every order in both
# precisions; meshes one element wider than a whole number of x and y tiles
# (ragged tiles, the element index n_d alone in a tile), small targets giving
# chunks of several element layers along z, and the default target
BITS = (1 << 0) | (1 << 4) | (1 << 8) | (1 << 9) | (1 << 12) | (1 << 16)
CASES = []
for _P in range(1, 9):
    for _word in (4, 8):
        _D = dims(_P, _word)
        _n = (_D["EX"] + 1, _D["EY"] + 1, 7)
        CASES.append((_P, _word, _n, BITS, 3 * 2 * 2 * 3))
        CASES.append((_P, _word, (max(1, _D["EX"] // 2), 2, 3), 0, 1024))
CASES += [(1, 4, (70, 3, 3), 0, 40), (4, 8, (17, 5, 6), (1 << 1) | (1 << 9), 16),
          (3, 4, (22, 9, 5), (1 << 12) | (1 << 16) | (1 << 4), 20)]


@pytest.mark.parametrize("P,word,n_el,bits,target", CASES)
def test_mass_stencil_decomposition(P, word, n_el, bits, target):
    rng = np.random.default_rng(100 + P)
    A = rng.standard_normal((P + 1, P + 1))
    Mq = A @ A.T + (P + 1) * np.eye(P + 1)
    Nn = (n_el[0] * P + 1) * (n_el[1] * P + 1) * (n_el[2] * P + 1)
    v = rng.standard_normal(3 * Nn)
    y, writes = run_model(P, word, n_el, Mq, v, bits, 1.7, target)
    assert np.array_equal(writes, np.ones(3 * Nn, dtype=int))
    ref = reference(P, n_el, Mq, v, bits, 1.7)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
