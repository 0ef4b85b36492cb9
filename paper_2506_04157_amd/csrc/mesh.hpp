// Host-side geometry: macro meshes, structured refinement, global numbering.
//
// Macro meshes follow Sec. 4.1 of arXiv 2506.04157 (hybrid hierarchical grid:
// unstructured macro-tetrahedra, each refined uniformly into 8^L micro-tets;
// the hollow sphere is built from the hollow icosahedron, cut into radial
// layers of equal height, each prism cut into three tetrahedra).  Where the
// paper is silent the same readings as the oracle are implemented here from
// their statement (icosahedron orientation, lexicographic order of the
// integer point keys, prism split, octahedron diagonal, radial blending).
//
// Global numbering: every P1/P2 node belongs to exactly one primitive of the
// macro mesh (vertex, edge, face or cell interior) and vectors are laid out
// [cell interiors | face interiors | edge interiors | vertices].  Per level and
// macro a local-to-global table maps the macro's lattice points
// (I,J,K), I+J+K <= m, in the order K-major, then J, then I, to global ids.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace stk {

enum { BC_NONE = 0, BC_DIRICHLET = 1, BC_FREESLIP = 2 };

struct MacroMesh {
  int kind = 0;                       // 0 cube, 1 shell
  double r_in = 0, r_out = 0;
  int n_rad = 0;
  std::vector<double> V;              // 3 * nv reference coordinates
  std::vector<int> layer;             // radial layer per vertex (shell)
  std::vector<std::array<int, 4>> tets;
  int nv() const { return (int)layer.size(); }
  int nm() const { return (int)tets.size(); }
};

MacroMesh make_cube();
MacroMesh make_shell(int n_tan, int n_rad, double r_in, double r_out);
// The unit icosahedron of the shell: 12 vertices and the 20 faces (vertex
// ids ascending, in the order make_shell refines them; face f's lattice
// point (i, j) has the weights i, j, n_tan - i - j on its vertices 0, 1, 2).
void icosahedron(double ico[12][3], std::vector<std::array<int, 3>>& faces);

// Number of lattice points with i+j+k <= s.
inline int64_t tet_count(int64_t s) { return s < 0 ? 0 : (s + 1) * (s + 2) * (s + 3) / 6; }
// Local index of lattice point (I,J,K) in a lattice of side m.
inline int64_t lattice_loc(int I, int J, int K, int m) {
  int s = m - K;
  return tet_count(m) - tet_count(m - K) + (int64_t)J * (s + 1) - (int64_t)J * (J - 1) / 2 + I;
}

// Primitives of the macro mesh and boundary classification.
struct Topology {
  std::vector<std::array<int, 3>> faces;   // sorted global vertex ids
  std::vector<std::array<int, 2>> edges;   // sorted
  std::vector<std::array<int, 4>> mface;   // per macro: global face id opposite local vertex f
  std::vector<std::array<int, 6>> medge;   // per macro: global edge id of local edge e
  std::vector<int> vkind, ekind, fkind;    // boundary kind: 0 interior, 1 inner/cube, 2 outer
  std::vector<int> vowner, eowner, fowner; // smallest macro containing the primitive
  std::vector<uint8_t> bkind;              // per macro x 16 (nonzero-weight mask): boundary kind
  std::vector<uint8_t> own;                // per macro x 16: 1 if this macro owns the sub-simplex
};

Topology build_topology(const MacroMesh& mm);

// One refinement level: numbering and per-macro tables.
struct Level {
  int L = 0, n = 1;                        // n = 2^L
  int64_t n2 = 0, n1 = 0;                  // global P2 / P1 node counts
  int64_t nloc2 = 0, nloc1 = 0;            // lattice points per macro
  std::vector<uint32_t> l2g2, l2g1;        // nm * nloc
  std::vector<uint32_t> bnode;             // boundary P2 nodes (each once)
  std::vector<uint8_t> bkind;              // their boundary kind (1 inner/cube, 2 outer)
  std::vector<double> bnormal;             // 3 per boundary node: x~/|x~| (radial normal)
  std::vector<double> tinv;                // nm * 6 types * 10: grad lambda_1..3 rows, |det J_F|
  std::vector<int> tiles;                  // brick origins (3 ints each) in the cube lattice
};

constexpr int TILE = 4;                    // cubes per brick side

// Plane-sweep decomposition of one macro-tet (the same for every macro of a
// level): the cube rows py are split into strips; a workgroup sweeps one
// (macro, strip) layer by layer along the third lattice direction.  Nodes on
// the macro boundary or on a strip boundary row are "shared": their partial
// sums go to per-(macro, strip, node) slots that a gather pass adds up.
struct Sweep {
  int nstrips = 1;
  std::vector<int> strip;      // j0, j1 (cube rows [j0, j1)) per strip
  // P2 / P1 plane lists per (strip, plane): entries (packed I | J<<10 | K<<20, slot or -1)
  std::vector<int> plist2, poff2, plist1, poff1;
  // elements per (strip, layer): packed type | px<<3 | py<<13
  std::vector<int> elist, eoff;
  // per element (same order as elist), 8 ints: the LDS ring positions of its
  // 10 P2 nodes (16 bits each, vertices then edges 01,02,03,12,13,23; words
  // 0-4), of its 4 P1 vertices (words 5-6), and its type (word 7).  P2 plane K
  // lives in ring slot K % 3 (cap2 entries each), P1 plane k in slot k % 2.
  std::vector<int> etab;
  int nsh2 = 0, nsh1 = 0;      // shared slots per macro
  int cap2 = 0, cap1 = 0;      // largest plane list (LDS ring slot size)
};
Sweep build_sweep(int n, int nstrips);
// Gather lists of the shared nodes: for each shared global node, the slots
// (macro * nsh + slot) holding its partial sums.  which = 2 (P2) or 1 (P1).
void build_gather(const MacroMesh& mm, const Level& lv, const Sweep& sw, int which, std::vector<uint32_t>& node,
                  std::vector<int>& ptr, std::vector<int>& slot);

// Lattice tables of the P1 mass stencil of one level (the same for every
// macro): a P1 lattice node couples with itself and its 14 lattice
// neighbours; direction 0 is the node itself, 1..7 the lexicographically
// positive lattice directions and 8..14 their negatives (d + 7 = -d).
constexpr int NDIR1 = 15;
struct P1Stencil {
  int dir[NDIR1][3];           // lattice offset of each direction
  std::vector<int16_t> nb;     // [NDIR1][nloc1] neighbour local index, nloc1 where absent
  std::vector<int> dst;        // [nloc1] slot of macro-boundary nodes, -1 for macro-interior ones
  std::vector<int> inc_ptr;    // [nloc1 + 1] micro-tets containing each node
  std::vector<int> inc;        // pairs: packed type | px<<3 | py<<13 | pz<<23, and
                               //        vertex v | (direction of vertex w) << (2 + 4 w)
  int nsh = 0;                 // slots per macro
  Sweep slots;                 // one-strip sweep whose P1 slots the stencil shares
};
P1Stencil build_p1_stencil(int n);

// Grid-transfer table of a coarse level (the same for every macro): for each
// brick (tile) of the coarse level, the fine P2 lattice points it handles, in
// lattice order, with the coarse P2 nodes whose basis functions are nonzero
// there.  8 ints per entry: fine point I | J<<10 | K<<20; number of nonzero
// weights (<= 10); five words of two 16-bit fields (brick-local coarse node
// index, 10 bits | (8 * weight + 1) << 10), in the coarse micro-tet's node
// order; padding.
struct TransferTable {
  // per tile: the fine points of its coarse cubes, those inside the macro
  // first (their global index is closed-form), each as 8 ints: packed
  // position, weight count, 5 words of two (brick index | (8 w + 1) << 10)
  std::vector<int> tab;
  std::vector<int> off;   // per tile: first entry (ntiles + 1)
};
TransferTable build_transfer_table(const Level& coarse);

Level build_level(const MacroMesh& mm, const Topology& top, int L);
// Blended coordinates (3 per node, nullable) and boundary kinds (nullable) of
// the P2 (which = 2) or P1 (which = 1) nodes of a level.
void level_coords(const MacroMesh& mm, const Topology& top, const Level& lv, int which, double* X,
                  uint8_t* flags);

// Per-macro geometry: v0(3), E columns (9: E[r*3+c] = (v_{c+1}-v0)_r), g(3), s0.
std::vector<double> macro_geometry(const MacroMesh& mm);

// Micro-tet type tables (lattice offsets of the 4 vertices, P1 units).
extern const int TYPE_OFF[6][4][3];
extern const int EDGE_V[6][2];

}  // namespace stk
