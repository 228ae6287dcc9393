// Host-side checks of libsoptx under AddressSanitizer and
// UndefinedBehaviorSanitizer: the pattern and plan builder, the mesh
// validation, the reference tensors and the filter builder, built from the
// library's own sources with g++ and run on meshes the test writes.
//
// Only host functions are called.  The device launchers that the same
// translation units reference stay unresolved at link time
// (--unresolved-symbols=ignore-all): none of the calls below reaches them.
//
// Usage: sanitize_host FILE...   each FILE holds int32 elem, dim, then int64
// n_nodes, n_cells, then n_nodes*dim doubles and n_cells*nen int32.
// Prints the status of every call, one line per file (the test checks them);
// a sanitizer finding aborts the process with a report and a nonzero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../include/soptx.h"
#include "../include/soptx_debug.h"

static const char *kArrays[] = {"row_ptr",  "col_idx",       "geo",       "sig_info",  "sig_pos_ptr",
                                "sig_contrib", "sig_pairs",  "sig_witems", "sig_witem_ptr", "grp_info",
                                "grp_nodes", "grp_elems",    "grp_n2l",   "grp_rows",  "grp_rank_off", "grp_rank", "elem_by_rank", "pos",
                                "nb_tslot",  "nb_tdeg",      "gptr",      "gent",      "gnode"};

static int nen_of(int elem) {
    switch (elem) {
    case SOPTX_QUAD4: return 4;
    case SOPTX_TRI3: return 3;
    case SOPTX_HEX8: return 8;
    case SOPTX_TET10: return 10;
    case SOPTX_HEX27: return 27;
    default: return -1;
    }
}

// touch every byte of every plan array (a read past the end is a finding)
static long long walk_plan(soptx_host_plan p) {
    long long sum = 0;
    for (const char *name : kArrays) {
        const void *data = nullptr;
        int64_t count = 0;
        int32_t eb = 0;
        if (soptx_debug_host_plan_array(p, name, &data, &count, &eb) != SOPTX_OK) continue;
        const unsigned char *b = static_cast<const unsigned char *>(data);
        for (int64_t i = 0; i < count * eb; i++) sum += b[i];
    }
    int64_t sc[8];
    soptx_debug_host_plan_scalars(p, sc);
    return sum + sc[0];
}

int main(int argc, char **argv) {
    for (int a = 1; a < argc; a++) {
        FILE *fh = std::fopen(argv[a], "rb");
        if (!fh) { std::printf("%s: cannot open\n", argv[a]); return 2; }
        int32_t hdr[2];
        int64_t sz[2];
        if (std::fread(hdr, 4, 2, fh) != 2 || std::fread(sz, 8, 2, fh) != 2) { std::fclose(fh); return 2; }
        const int elem = hdr[0], dim = hdr[1], nen = nen_of(elem);
        std::vector<double> coords((size_t)sz[0] * dim);
        std::vector<int32_t> cells((size_t)sz[1] * (nen > 0 ? nen : 0));
        if (std::fread(coords.data(), 8, coords.size(), fh) != coords.size() ||
            std::fread(cells.data(), 4, cells.size(), fh) != cells.size()) {
            std::fclose(fh);
            return 2;
        }
        std::fclose(fh);
        soptx_mesh m{};
        m.elem = elem;
        m.dim = dim;
        m.n_nodes = sz[0];
        m.n_cells = sz[1];
        m.coords = coords.data();
        m.cells = cells.data();
        const int v = soptx_validate_mesh(&m);
        long long touched = 0;
        int plan_rc[2] = {0, 0};
        for (int general = 0; general < 2; general++) {
            soptx_host_plan p = nullptr;
            plan_rc[general] = soptx_debug_host_plan_ex(&m, general, &p);
            if (plan_rc[general] == SOPTX_OK) {
                touched += walk_plan(p);
                soptx_debug_host_plan_free(p);
            }
        }
        int64_t fn = 0, fnnz = 0;
        int frc = soptx_debug_filter_matrix(&m, dim == 2 ? 2.5 : 1.5, &fn, &fnnz, nullptr, nullptr, nullptr,
                                            nullptr, nullptr, nullptr);
        if (frc == SOPTX_OK && fnnz > 0) {
            std::vector<int32_t> rp((size_t)fn + 1), col((size_t)fnnz);
            std::vector<double> w((size_t)fnnz), vol((size_t)fn), hsv((size_t)fn), hs((size_t)fn);
            frc = soptx_debug_filter_matrix(&m, dim == 2 ? 2.5 : 1.5, &fn, &fnnz, rp.data(), col.data(), w.data(),
                                            vol.data(), hsv.data(), hs.data());
            for (int64_t k = 0; k < fnnz; k++) touched += col[(size_t)k];
        }
        int32_t S = 0;
        int64_t N[3] = {0, 0, 0};
        const int src = soptx_debug_filter_stencil(&m, dim == 2 ? 2.5 : 1.5, &S, N);
        int rrc = 0;
        if (nen > 0) {
            std::vector<double> M((size_t)nen * nen * dim * dim);
            for (int method = 0; method < 2; method++) rrc |= soptx_reference_tensor(elem, method, M.data());
        }
        std::printf("%s: validate %d plan %d general %d filter %d stencil %d(%d) reference %d touched %lld\n",
                    argv[a], v, plan_rc[0], plan_rc[1], frc, src, S, rrc, touched % 1000);
    }
    return 0;
}
