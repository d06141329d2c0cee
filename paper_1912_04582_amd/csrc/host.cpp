// Host-only checks of the library (mesh validation, checkpoint buffers); no
// HIP, so that they can also be built and exercised on their own.
#include <cmath>
#include <cstring>

#include "tk_host.h"

int face_axis(const double* e) {
  int axis = -1, nz = 0;
  for (int a = 0; a < 3; ++a)
    if (e[a] != 0.0) { axis = a; ++nz; }
  return (nz == 1 && std::fabs(std::fabs(e[axis]) - 1.0) <= 1e-12) ? axis : -1;
}

namespace tk {

static tk_status fail(std::string* err, const std::string& msg) {
  if (err) *err = msg;
  return TK_EINVAL;
}

tk_status mesh_build_host(const tk_mesh_desc* d, tk_mesh* m, std::string* err) {
  if (!d || !m || d->n_cells <= 0 || d->n_faces <= 0 || !d->face_left || !d->face_right || !d->face_normal ||
      !d->face_area || !d->cell_volume || d->n_bc < 0 || (d->n_bc > 0 && !d->bc))
    return fail(err, "mesh: missing arrays or empty mesh");
  const int nc = d->n_cells, nf = d->n_faces;
  m->n_cells = nc;
  m->n_faces = nf;
  m->volume.assign(d->cell_volume, d->cell_volume + nc);
  m->bc.assign(d->bc, d->bc + d->n_bc);
  for (int i = 0; i < nc; ++i)
    if (!(m->volume[i] > 0.0) || !std::isfinite(m->volume[i]))
      return fail(err, "mesh: non-positive cell volume at cell " + std::to_string(i));
  for (const tk_bc& b : m->bc)
    if (b.kind < TK_BC_SYM || b.kind > TK_BC_WALL) return fail(err, "mesh: unknown bc kind");
  m->slot_nb.assign((size_t)nc * kSlots, -1);
  m->slot_kind.assign((size_t)nc * kSlots, SK_NONE);
  m->slot_axis.assign((size_t)nc * kSlots, 0);
  m->slot_sig.assign((size_t)nc * kSlots, 1);
  m->slot_area.assign((size_t)nc * kSlots, 0.0);
  m->slot_l1.assign((size_t)nc * kSlots, 0.0);
  m->slot_nrm.assign((size_t)nc * kSlots * 3, 0.0);
  m->slot_face.assign((size_t)nc * kSlots, -1);
  m->face_normal.assign(d->face_normal, d->face_normal + 3 * (size_t)nf);
  m->oblique = false;
  std::vector<int> cnt(nc, 0);
  int cur_face = -1;
  std::vector<double> close((size_t)nc * 3, 0.0), asum(nc, 0.0);
  auto add_slot = [&](int c, int nb, int8_t kind, const double* e, double sgn, double A) -> tk_status {
    if (cnt[c] >= kSlots) return fail(err, "mesh: cell " + std::to_string(c) + " has more than 6 faces");
    int axis = face_axis(e);
    const bool on_axis = axis >= 0;
    if (!on_axis) {
      axis = -1;
      if (kind == SK_SYM || kind == SK_WALL)
        return fail(err, "mesh: symmetry and wall faces must lie on coordinate-axis planes");
      m->oblique = true;
    }
    const int s = cnt[c]++;
    const size_t k = (size_t)c * kSlots + s;
    m->slot_nb[k] = nb;
    m->slot_kind[k] = kind;
    m->slot_axis[k] = (int8_t)axis;
    m->slot_sig[k] = (int8_t)((on_axis ? sgn * e[axis] : sgn) > 0 ? 1 : -1);
    for (int a = 0; a < 3; ++a) m->slot_nrm[3 * k + a] = sgn * e[a];
    m->slot_face[k] = cur_face;
    m->slot_area[k] = A;
    m->slot_l1[k] = A * (std::fabs(e[0]) + std::fabs(e[1]) + std::fabs(e[2]));
    for (int a = 0; a < 3; ++a) close[3 * c + a] += sgn * A * e[a];
    asum[c] += A;
    return TK_OK;
  };
  for (int j = 0; j < nf; ++j) {
    cur_face = j;
    const int L = d->face_left[j], R = d->face_right[j];
    const double* e = d->face_normal + 3 * (size_t)j;
    const double A = d->face_area[j];
    if (L < 0 || L >= nc) return fail(err, "mesh: face_left out of range at face " + std::to_string(j));
    if (!(A > 0.0) || !std::isfinite(A)) return fail(err, "mesh: bad face area");
    const double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!(std::fabs(en - 1.0) <= 1e-10)) return fail(err, "mesh: face normal is not unit length");
    tk_status st;
    if (R >= 0) {
      if (R >= nc || R == L) return fail(err, "mesh: face_right out of range");
      if ((st = add_slot(L, R, SK_INTERIOR, e, 1.0, A)) != TK_OK) return st;
      if ((st = add_slot(R, L, SK_INTERIOR, e, -1.0, A)) != TK_OK) return st;
    } else {
      // boundary index -R - 1, computed without overflowing at INT_MIN
      const long long b = -(long long)R - 1;
      if (b >= (long long)m->bc.size()) return fail(err, "mesh: boundary index out of range");
      int8_t kind = SK_NONE;
      switch (m->bc[b].kind) {
        case TK_BC_SYM: kind = SK_SYM; break;
        case TK_BC_INFLOW: kind = SK_INFLOW; break;
        case TK_BC_OUTFLOW: kind = SK_OUTFLOW; break;
        case TK_BC_WALL: kind = SK_WALL; break;
      }
      if ((st = add_slot(L, (int)b, kind, e, 1.0, A)) != TK_OK) return st;
    }
  }
  for (int c = 0; c < nc; ++c) {
    const double r = std::sqrt(close[3 * c] * close[3 * c] + close[3 * c + 1] * close[3 * c + 1] +
                               close[3 * c + 2] * close[3 * c + 2]);
    if (!(r <= 1e-12 * asum[c])) return fail(err, "mesh: cell " + std::to_string(c) + " is not closed");
  }
  return TK_OK;
}

tk_status ckpt_check_header(const void* buf, size_t bytes, const CkptHeader& want, size_t total,
                            std::string* err) {
  if (!buf || bytes < sizeof(CkptHeader)) return fail(err, "restore: buffer too small");
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "TKCKPT2", 8) != 0) return fail(err, "restore: not a checkpoint");
  if (h.N != want.N || h.CS != want.CS || h.nc != want.nc || h.ninst != want.ninst || h.mixed != want.mixed ||
      h.plain != want.plain)
    return fail(err, "restore: checkpoint of a different state shape");
  if (bytes < total) return fail(err, "restore: buffer too small");
  return TK_OK;
}

tk_status ckpt_check_ranks(const int* rank, size_t n, int CS, std::string* err) {
  for (size_t i = 0; i < n; ++i)
    if (rank[i] < 1 || rank[i] > CS)
      return fail(err, "restore: rank " + std::to_string(rank[i]) + " out of 1.." + std::to_string(CS) +
                           " at entry " + std::to_string(i));
  return TK_OK;
}

}  // namespace tk
