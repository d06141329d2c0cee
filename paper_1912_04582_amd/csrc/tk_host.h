// Host-only parts of the library, free of HIP: the constants of the face
// slots, the mesh object and its validation, and the checks of checkpoint
// buffers.  Compiled into libtk (host.cpp) and, on their own, into a
// sanitizer build of those checks.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "tk.h"

namespace tk {

constexpr int kMaxCap = 16;  // largest Tucker rank per mode
constexpr int kSlots = 6;    // faces per hexahedral cell

// Kind of the cell on the far side of a face slot.
enum SlotKind : int8_t {
  SK_NONE = -1,     // unused slot (cell with fewer than 6 faces)
  SK_INTERIOR = 0,  // another cell of the same state
  SK_INFLOW = 1,    // free-stream Maxwellian
  SK_OUTFLOW = 2,   // zero-gradient: the cell itself
  SK_SYM = 3,       // symmetry plane: the cell with one velocity axis reversed
  SK_WALL = 4,      // diffuse wall: n_w times the unit wall Maxwellian
};

// Fixed part of a checkpoint buffer (tk_state_checkpoint).
struct CkptHeader {
  char magic[8];  // "TKCKPT2"
  int32_t N, CS, nc, ninst, mixed, plain, warm, pad;
};

}  // namespace tk

// the coordinate axis a unit face normal lies on, or -1 (an oblique face)
int face_axis(const double* e);

struct tk_mesh {
  tk_ctx* ctx = nullptr;
  int n_cells = 0, n_faces = 0;
  std::vector<double> volume;
  std::vector<tk_bc> bc;
  // per cell, kSlots face slots
  std::vector<int> slot_nb;        // neighbour cell or local bc index
  std::vector<int8_t> slot_kind;   // tk::SlotKind
  std::vector<int8_t> slot_axis;
  std::vector<int8_t> slot_sig;    // outward orientation along the axis
  std::vector<double> slot_area;
  std::vector<double> slot_l1;     // A ||e||_1
  std::vector<double> slot_nrm;    // [nc][6][3] outward unit normal
  std::vector<int> slot_face;      // face index of the slot
  bool oblique = false;            // some face normal is off the coordinate axes
  std::vector<double> face_normal; // [n_faces][3]
};

namespace tk {

// Validates a mesh description and builds the per-cell face slots into m:
// arrays present, counts positive, volumes and areas positive and finite,
// unit normals, face and boundary indices in range, at most six faces per
// cell, symmetry and wall faces on coordinate-axis planes, every cell closed
// (|sum_l s_l A_l e_l| <= 1e-12 sum_l A_l).  TK_EINVAL with a message in
// *err otherwise.
tk_status mesh_build_host(const tk_mesh_desc* d, tk_mesh* m, std::string* err);

// A checkpoint buffer of `bytes` bytes against the state it is restored
// into: its header (magic and shape fields equal to `want`'s) and its size
// (at least `total`).
tk_status ckpt_check_header(const void* buf, size_t bytes, const CkptHeader& want, size_t total,
                            std::string* err);

// Restored ranks: every entry of rank[n] in 1..CS.
tk_status ckpt_check_ranks(const int* rank, size_t n, int CS, std::string* err);

}  // namespace tk
