// Host-only shim around the general-mesh analysis of the library (no GPU):
// runs analyse_general and hands its tables to the CPU tests.
#include <cstring>

#include "../paper_1509_01399_amd/csrc/hyb_gen.h"

static hyb::GenHost g_tab;
static std::string g_err;

extern "C" int gen_analyse(const hyb_fd_grid *gr, const hyb_fem_mesh *m, const int *o, const int *C,
                           long long *sizes)
{
    g_tab = hyb::GenHost();
    const int st = (int)hyb::analyse_general(gr, m, o, C, g_tab, g_err);
    if (st) return st;
    const long long v[] = {g_tab.fn, g_tab.nA, g_tab.nH, g_tab.nR, g_tab.ntet, g_tab.nslice, g_tab.nslice_h,
                           g_tab.nnz, g_tab.nE, g_tab.nedge, (long long)g_tab.cw.size(), g_tab.all_grid ? 1 : 0};
    std::memcpy(sizes, v, sizeof v);
    return 0;
}

extern "C" const char *gen_error() { return g_err.c_str(); }

template <typename V>
static void put(void *dst, const std::vector<V> &src)
{
    if (!src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(V));
}

// Copy one table (by name) into dst, sized from gen_analyse.
extern "C" int gen_table(const char *name, void *dst)
{
    const std::string n(name);
    if (n == "orig_of_dev") put(dst, g_tab.orig_of_dev);
    else if (n == "grid_lin") put(dst, g_tab.grid_lin);
    else if (n == "gq") put(dst, g_tab.gq);
    else if (n == "soff") put(dst, g_tab.soff);
    else if (n == "eoff") put(dst, g_tab.eoff);
    else if (n == "col") put(dst, g_tab.col);
    else if (n == "eid") put(dst, g_tab.eid);
    else if (n == "cptr") put(dst, g_tab.cptr);
    else if (n == "ctet") put(dst, g_tab.ctet);
    else if (n == "cw") put(dst, g_tab.cw);
    else if (n == "minv") put(dst, g_tab.minv);
    else if (n == "tetE") put(dst, g_tab.tetE);
    else if (n == "ke6") put(dst, g_tab.ke6);
    else if (n == "pvol") put(dst, g_tab.pvol);
    else return -1;
    return 0;
}
