"""Force models (oracle, float64, plain PyTorch CPU ops).

Two models are evaluated on a CSR neighbour list (see ``neighbors``):

1. The conservative potential U (paper, Methods "Model architecture", first
   paragraph: an embedding refined by equivariant message passing, atomic
   energies from perceptrons, E = sum_i E_i, forces = -grad E).  The paper's
   FeNNix-Bio1(M) weights and exact layers are not available, so this is a
   synthetic l <= 1 equivariant message-passing model of the same kind
   (species embedding, Bessel radial filter with a cosine cutoff, scalar and
   vector features, SiLU perceptrons).  Per layer, with every term using the
   layer-input features (a synchronous update):

       phi_j          = W2 silu(W1 s_j + b1) + b2                 in R^{3F}
       w_ij           = (Wr e(r_ij) + br) fcos(r_ij)               in R^{3F}
       [a|b|c]_ij     = phi_j * w_ij
       s_i           += sum_j a_ij
       v_i[alpha]    += sum_j (b_ij * v_j[alpha] + u_ij[alpha] c_ij)
     then the update block
       Uv = U v, Vv = V v (per Cartesian component, no bias)
       n  = sqrt(sum_alpha Vv[alpha]^2 + 1e-8)
       [p|q|o] = M2 silu(M1 [s; n] + m1) + m2
       s += p + q * sum_alpha Uv[alpha] * Vv[alpha]
       v[alpha] += o * Uv[alpha]
     readout  E_i = wo . silu(Wo s_i + bo) + beta[t_i].

   Forces are -dE/dx from torch.autograd (a library routine).

2. The distilled non-conservative force model (paper, Methods, equations for
   q_ih, k_ih, c_ijh, F_ij and F_i): one embedding layer of the block above
   at the short-range cutoff with the polynomial envelope, then
       q_ih = Wq[h] s_i,  k_ih = Wk[h] s_i                  (n_c each)
       V_ih = sum_f WV[h, f] v_i[:, f]                        (vector heads)
       c_ijh = (q_ih . k_jh) / sqrt(n_c)
       F_ij = (sum_{h<=n_s} c_ijh B_h(r_ij))
              (u_ij + sum_{h<=n_l} c_ij(n_s+h) V_ih) f_c(r_ij)
       F_i  = sum_{j in N(i)} (F_ij - F_ji)
   The screened nuclear repulsion term is off (its parameters are not
   available); ``nc_forces`` takes no repulsion.

3. Virials for NPT (paper, Methods "Computation of the virial term in NPT"):
   the quantity W = -sum_i F_i . q_i, written under periodic boundaries
   through the minimum-image vectors r_ij = q_j - q_i.
   * Conservative model: W = sum over directed edges of r_e . dE/dr_e, which
     is dE(lambda)/dlambda at lambda = 1 when every position and the box are
     scaled by lambda (all minimum-image vectors scale with lambda); taken
     by autograd in lambda.
   * NC model: the paper's proxy W = sum_i sum_{j in N(i)} F_ij . r_ij.

Shared pieces:
   Bessel basis  e_k(r) = sqrt(2/rc) sin(k pi r / rc) / r,  k = 1..K
   cosine cutoff fcos(r) = (cos(pi r / rc) + 1) / 2 for r < rc, else 0
   polynomial envelope (order p) with d = r / rc:
       u(d) = 1 - (p+1)(p+2)/2 d^p + p(p+2) d^{p+1} - p(p+1)/2 d^{p+2}, d < 1
   u_ij = r_ij / |r_ij| with r_ij = x_j - x_i under the minimum image.

Weight vectors are flat float64 arrays in the manifest order documented with
the C interface ([out][in] row-major matrices).

Pins (tests/test_oracle_models.py): closed forms of the basis and cutoffs;
forces against central finite differences of the energy; invariance of E
under translation, the cubic symmetries of the box, same-species permutation
and rotation of an isolated cluster; additivity of E over clusters beyond the
cutoff; continuity of E as a pair crosses the cutoff; reduction to per-atom
perceptrons (evaluated with torch.nn.functional.linear) when the radial filter
is a constant; NC forces summing to zero over each connected component,
rotation equivariance, central pair forces with a symmetric weight when there
are no vector heads, zero forces for zero queries, a closed form of the pair
force of a two-species dimer with hand-set weights (which tells the owner's
vector heads V_i from the neighbour's and c_ijh = q_ih . k_jh from q_jh . k_ih),
and the weight gradient against finite differences.
"""

import math

import numpy as np
import torch
import torch.nn.functional as tF

from .neighbors import edge_index

_F64 = torch.float64


# ----------------------------------------------------------------- weights --

def _block_layout(prefix, F, K):
    return [
        (prefix + "W1", (F, F)), (prefix + "b1", (F,)),
        (prefix + "W2", (3 * F, F)), (prefix + "b2", (3 * F,)),
        (prefix + "Wr", (3 * F, K)), (prefix + "br", (3 * F,)),
        (prefix + "U", (F, F)), (prefix + "V", (F, F)),
        (prefix + "M1", (F, 2 * F)), (prefix + "m1", (F,)),
        (prefix + "M2", (3 * F, F)), (prefix + "m2", (3 * F,)),
    ]


def layout(spec):
    """(name, shape) in manifest order for a conservative or NC model."""
    F, K, S = spec.width, spec.n_rbf, spec.n_species
    out = [("emb", (S, F))]
    if spec.kind == "cons":
        for layer in range(spec.n_layers):
            out += _block_layout(f"l{layer}.", F, K)
        out += [("Wo", (F, F)), ("bo", (F,)), ("wo", (1, F)), ("beta", (S,))]
    else:
        H = spec.n_s + spec.n_l
        out += _block_layout("l0.", F, K)
        out += [("Wq", (H, spec.n_c, F)), ("Wk", (H, spec.n_c, F)), ("WV", (spec.n_l, F))]
    return out


def unpack(spec, theta):
    """Split a flat weight tensor into named views."""
    theta = torch.as_tensor(theta, dtype=_F64) if not torch.is_tensor(theta) else theta
    p, k = {}, 0
    for name, shape in layout(spec):
        size = int(np.prod(shape))
        p[name] = theta[k:k + size].reshape(shape)
        k += size
    if k != theta.numel():
        raise ValueError(f"weight vector has {theta.numel()} entries, manifest needs {k}")
    return p


# ------------------------------------------------------------ radial parts --

def bessel(r, n, rc):
    """e_k(r) = sqrt(2/rc) sin(k pi r / rc) / r for k = 1..n  -> (E, n)."""
    k = torch.arange(1, n + 1, dtype=_F64)
    return math.sqrt(2.0 / rc) * torch.sin(k[None, :] * math.pi * r[:, None] / rc) / r[:, None]


def cosine_cutoff(r, rc):
    return torch.where(r < rc, 0.5 * (torch.cos(math.pi * r / rc) + 1.0), torch.zeros_like(r))


def poly_envelope(r, rc, p):
    d = r / rc
    u = (1.0 - (p + 1) * (p + 2) / 2.0 * d ** p + p * (p + 2) * d ** (p + 1)
         - p * (p + 1) / 2.0 * d ** (p + 2))
    return torch.where(d < 1.0, u, torch.zeros_like(r))


def edge_vectors(pos, box, i, j):
    """r_ij = x_j - x_i under the minimum image (differentiable in pos)."""
    d = pos[j] - pos[i]
    return d - box * torch.round(d * (1.0 / box)).detach()


# ------------------------------------------------------------- embedding ---

def _layer(p, prefix, s, v, i, j, ebasis, fcut, unit):
    F = s.shape[1]
    n = s.shape[0]
    phi = tF.silu(s @ p[prefix + "W1"].T + p[prefix + "b1"]) @ p[prefix + "W2"].T + p[prefix + "b2"]
    w = (ebasis @ p[prefix + "Wr"].T + p[prefix + "br"]) * fcut[:, None]
    msg = phi[j] * w
    a, b, c = msg[:, :F], msg[:, F:2 * F], msg[:, 2 * F:]
    ds = torch.zeros(n, F, dtype=_F64).index_add(0, i, a)
    dv = torch.zeros(n, 3, F, dtype=_F64).index_add(
        0, i, b[:, None, :] * v[j] + unit[:, :, None] * c[:, None, :])
    s = s + ds
    v = v + dv
    Uv = v @ p[prefix + "U"].T
    Vv = v @ p[prefix + "V"].T
    nrm = torch.sqrt((Vv * Vv).sum(dim=1) + 1e-8)
    h = tF.silu(torch.cat([s, nrm], dim=1) @ p[prefix + "M1"].T + p[prefix + "m1"]) \
        @ p[prefix + "M2"].T + p[prefix + "m2"]
    pp, qq, oo = h[:, :F], h[:, F:2 * F], h[:, 2 * F:]
    s = s + pp + qq * (Uv * Vv).sum(dim=1)
    v = v + oo[:, None, :] * Uv
    return s, v


def _geometry(spec, pos, box, offsets, nbr):
    i, j = edge_index(offsets, nbr)
    i = torch.as_tensor(i)
    j = torch.as_tensor(j)
    rvec = edge_vectors(pos, box, i, j)
    r = torch.sqrt((rvec * rvec).sum(dim=1))
    unit = rvec / r[:, None]
    ebasis = bessel(r, spec.n_rbf, spec.cutoff)
    if spec.kind == "cons":
        fcut = cosine_cutoff(r, spec.cutoff)
    else:
        fcut = poly_envelope(r, spec.cutoff, spec.poly_p)
    return i, j, r, unit, ebasis, fcut


def embed(spec, p, pos, species, box, offsets, nbr):
    """Scalar and vector features (s (N,F), v (N,3,F)) after all layers."""
    i, j, r, unit, ebasis, fcut = _geometry(spec, pos, box, offsets, nbr)
    sp = torch.as_tensor(np.asarray(species, dtype=np.int64))
    s = p["emb"][sp]
    v = torch.zeros(s.shape[0], 3, s.shape[1], dtype=_F64)
    n_layers = spec.n_layers if spec.kind == "cons" else 1
    for layer in range(n_layers):
        s, v = _layer(p, f"l{layer}.", s, v, i, j, ebasis, fcut, unit)
    return s, v, (i, j, r, unit)


# ----------------------------------------------------------- conservative --

def cons_atomic_energies(spec, theta, pos, species, box, offsets, nbr):
    p = unpack(spec, theta)
    s, _, _ = embed(spec, p, pos, species, box, offsets, nbr)
    sp = torch.as_tensor(np.asarray(species, dtype=np.int64))
    return (tF.silu(s @ p["Wo"].T + p["bo"]) @ p["wo"].T)[:, 0] + p["beta"][sp]


def cons_energy(spec, theta, pos, species, box, offsets, nbr):
    """E = sum_i E_i (kcal/mol) as a float."""
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    with torch.no_grad():
        return float(cons_atomic_energies(spec, theta, x, species, box, offsets, nbr).sum())


def cons_energy_forces(spec, theta, pos, species, box, offsets, nbr):
    """(E, F) with F = -dE/dx, (N, 3) float64 numpy."""
    x = torch.tensor(np.asarray(pos, dtype=np.float64), requires_grad=True)
    e = cons_atomic_energies(spec, theta, x, species, box, offsets, nbr).sum()
    (g,) = torch.autograd.grad(e, x)
    return float(e.detach()), (-g).numpy()


def cons_virial(spec, theta, pos, species, box, offsets, nbr):
    """W = -sum_i F_i . q_i = dE/dlambda under q -> lambda q, L -> lambda L
    (minimum-image vectors scale with lambda; images fixed), as a float."""
    lam = torch.tensor(1.0, dtype=_F64, requires_grad=True)
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    e = cons_atomic_energies(spec, theta, x * lam, species, torch.as_tensor(box, dtype=_F64) * lam,
                             offsets, nbr).sum()
    (g,) = torch.autograd.grad(e, lam)
    return float(g)


# -------------------------------------------------------- non-conservative --

def nc_pair_terms(spec, p, pos, species, box, offsets, nbr):
    """Per directed edge: F_ij (E, 3), plus the edge endpoints."""
    s, v, (i, j, r, unit) = embed(spec, p, pos, species, box, offsets, nbr)
    ns, nl, nc = spec.n_s, spec.n_l, spec.n_c
    q = torch.einsum("hcf,nf->nhc", p["Wq"], s)
    k = torch.einsum("hcf,nf->nhc", p["Wk"], s)
    V = torch.einsum("lf,naf->nla", p["WV"], v)
    c = (q[i] * k[j]).sum(dim=2) / math.sqrt(nc)
    B = bessel(r, ns, spec.cutoff)
    S = (c[:, :ns] * B).sum(dim=1)
    D = unit + (c[:, ns:ns + nl, None] * V[i]).sum(dim=1)
    fc = poly_envelope(r, spec.cutoff, spec.poly_p)
    Fij = S[:, None] * D * fc[:, None]
    return Fij, i, j


def nc_forces_t(spec, theta, pos, species, box, offsets, nbr):
    p = unpack(spec, theta)
    Fij, i, j = nc_pair_terms(spec, p, pos, species, box, offsets, nbr)
    n = pos.shape[0]
    zero = torch.zeros(n, 3, dtype=_F64)
    return zero.index_add(0, i, Fij) - zero.index_add(0, j, Fij)


def nc_forces(spec, theta, pos, species, box, offsets, nbr):
    """F_i = sum_j (F_ij - F_ji), (N, 3) float64 numpy."""
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    with torch.no_grad():
        return nc_forces_t(spec, theta, x, species, box, offsets, nbr).numpy()


def nc_virial_proxy(spec, theta, pos, species, box, offsets, nbr):
    """The NPT virial proxy sum_i sum_{j in N(i)} F_ij . r_ij (r_ij = q_j - q_i,
    minimum image), as a float."""
    p = unpack(spec, theta)
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    with torch.no_grad():
        Fij, i, j = nc_pair_terms(spec, p, x, species, box, offsets, nbr)
        rvec = edge_vectors(x, box, i, j)
        return float((Fij * rvec).sum())


def nc_weight_grad(spec, theta, pos, species, box, offsets, nbr, dl_df):
    """dL/dtheta for a loss whose gradient w.r.t. the NC forces is dl_df
    (N, 3): the vector-Jacobian product of the force model in its weights."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    f = nc_forces_t(spec, th, x, species, box, offsets, nbr)
    (g,) = torch.autograd.grad((f * torch.as_tensor(np.asarray(dl_df, dtype=np.float64))).sum(), th)
    return g.numpy()
