"""Lattice topology for the oracle (test infrastructure only).

Paper, Sec. "Model": a k x l rectangular lattice with open boundary
conditions, nearest-neighbour bonds.  Sec. "Pauli Basis Tensor Network":
deg(v) is 2 at corners, 3 on edges, 4 in the interior, and the site tensor
carries one bond leg per neighbour plus the Pauli leg.  Sec. "GPU Tensor
Permutation": legs are stored in the order [U, D, L, R, Pauli].
Sec. "Trotter Decomposition": bonds are split into four colour classes with
no shared site.  Sec. "Numerical Experiments": the observable sits at
(floor((Nx-1)/2), floor((Ny-1)/2)).

Numbering (an interface choice, identical in the C library but implemented
separately there):
  site id      v = x + Lx * y
  neighbours   U = (x, y-1), D = (x, y+1), L = (x-1, y), R = (x+1, y)
  bonds        all horizontal ((x,y),(x+1,y)) in row-major order, then all
               vertical ((x,y),(x,y+1)) in row-major order; v1 < v2
  colours      horizontal, x even -> 0; horizontal, x odd -> 1;
               vertical,   y even -> 2; vertical,   y odd -> 3
"""

LEG_NAMES = ("U", "D", "L", "R")


class Lattice:
    def __init__(self, Lx, Ly):
        if Lx < 1 or Ly < 1 or Lx * Ly < 2:
            raise ValueError("lattice needs Lx, Ly >= 1 and at least 2 sites")
        self.Lx, self.Ly = Lx, Ly
        self.n_sites = Lx * Ly
        self.bonds = []          # (v1, v2, orientation 'h' | 'v')
        self.colour = []
        for y in range(Ly):
            for x in range(Lx - 1):
                self.bonds.append((self.site(x, y), self.site(x + 1, y), "h"))
                self.colour.append(0 if x % 2 == 0 else 1)
        for y in range(Ly - 1):
            for x in range(Lx):
                self.bonds.append((self.site(x, y), self.site(x, y + 1), "v"))
                self.colour.append(2 if y % 2 == 0 else 3)
        self.n_bonds = len(self.bonds)
        bond_of = {}
        for b, (v1, v2, _) in enumerate(self.bonds):
            bond_of[(v1, v2)] = b
            bond_of[(v2, v1)] = b
        # legs[v]: list of (leg name, neighbour, bond id) in canonical U,D,L,R order
        self.legs = []
        for v in range(self.n_sites):
            x, y = self.coords(v)
            cand = (("U", x, y - 1), ("D", x, y + 1), ("L", x - 1, y), ("R", x + 1, y))
            lv = []
            for name, nx, ny in cand:
                if 0 <= nx < Lx and 0 <= ny < Ly:
                    u = self.site(nx, ny)
                    lv.append((name, u, bond_of[(v, u)]))
            self.legs.append(lv)

    def site(self, x, y):
        return x + self.Lx * y

    def coords(self, v):
        return v % self.Lx, v // self.Lx

    def degree(self, v):
        return len(self.legs[v])

    def centre(self):
        return self.site((self.Lx - 1) // 2, (self.Ly - 1) // 2)

    def leg_position(self, v, b):
        """Axis of site v's tensor that carries bond b."""
        for i, (_, _, bb) in enumerate(self.legs[v]):
            if bb == b:
                return i
        raise KeyError((v, b))

    def direction(self, b, src):
        """Directed-bond index: 0 for v1 -> v2, 1 for v2 -> v1."""
        v1, v2, _ = self.bonds[b]
        if src == v1:
            return 0
        if src == v2:
            return 1
        raise KeyError((b, src))

    def bonds_of_colour(self, c):
        return [b for b in range(self.n_bonds) if self.colour[b] == c]

    def manhattan(self, v, w):
        (x1, y1), (x2, y2) = self.coords(v), self.coords(w)
        return abs(x1 - x2) + abs(y1 - y2)
