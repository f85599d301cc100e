// CPU driver for the host-only parts of libfewfit -- the portability-tuning
// routines (ptune.cpp) and the descriptor, manifest and set-file parser
// (setfile.cpp) -- built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_sanitizers_cpu.py.  Any out-of-bounds access, use after
// free, leak, signed overflow or misaligned access aborts the run.
//
// usage: ptune_setfile_driver <sets dir> <variants dir> <scratch dir>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <random>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fewfit.h"
#include "../../paper_2507_15277_amd/csrc/setfile.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAIL: %s\n", what);
        ++failures;
    }
}

std::string slurp(const std::string& path)
{
    std::ifstream f(path, std::ios::binary);
    std::stringstream ss;
    ss << f.rdbuf();
    return ss.str();
}

void spit(const std::string& path, const std::string& text)
{
    std::ofstream f(path, std::ios::binary | std::ios::trunc);
    f << text;
}

// Every committed set file parses; every mutation of it either parses or is
// refused with FF_ERR_PARSE, and never touches memory it does not own.
void parser_cases(const std::string& sets, const std::string& variants, const std::string& scratch)
{
    std::vector<FfDesc> manifest;
    std::string err;
    expect(ff_read_manifest(variants.c_str(), manifest, err) == FF_OK && !manifest.empty(), "manifest parses");
    expect(ff_read_manifest((scratch + "/none").c_str(), manifest, err) == FF_ERR_IO, "missing manifest is FF_ERR_IO");
    const char* names[] = {"set_k1.txt", "set_k2.txt", "set_k4.txt", "set_k8.txt", "fixed_k1.txt",
                           "set_bf16x3_k4.txt", "set_bf16x6_k4.txt", "set_fp16s_k4.txt", "set_fp16x3_k4.txt",
                           "set_mixed_k4.txt"};
    std::mt19937_64 rng(2507);
    const std::string tmp = scratch + "/mutated_set.txt";
    long parsed = 0, refused = 0;
    for (const char* n : names) {
        const std::string path = sets + "/" + n;
        FfSetFile s;
        expect(ff_read_set_file(path.c_str(), s, err) == FF_OK, ("committed set parses: " + path).c_str());
        expect(s.cost.size() == s.shapes.size() * s.members.size(), "cost is ntrain x k");
        if (std::string(n) == "set_mixed_k4.txt") {
            // The mixed slot holds members of more than one precision form.
            bool several = false;
            for (const FfDesc& v : s.members) several = several || v.prec != s.members[0].prec;
            expect(s.form == kFfPrecForms && several, "mixed set: its own slot, members of several forms");
        }
        const std::string text = slurp(path);
        // Truncated at every byte, then random byte edits and token swaps.
        for (size_t cut = 0; cut < text.size(); cut += 1 + text.size() / 400) {
            spit(tmp, text.substr(0, cut));
            int rc = ff_read_set_file(tmp.c_str(), s, err);
            expect(rc == FF_OK || rc == FF_ERR_PARSE, "truncated file: parse or FF_ERR_PARSE");
            (rc == FF_OK ? parsed : refused)++;
        }
        const char* junk[] = {"-1", "0", "99999999999999999999", "nan", "inf", "-inf", "1e308", "x", "#", "\n",
                              "2147483648", "-2147483649", "variant", "rule", "end", "  ", "\t"};
        for (int t = 0; t < 300; ++t) {
            std::string m = text;
            const size_t at = rng() % (m.size() + 1);
            switch (rng() % 4) {
                case 0: m.insert(at, junk[rng() % (sizeof junk / sizeof *junk)]); break;
                case 1: if (at < m.size()) m[at] = (char)(rng() % 256); break;
                case 2: if (at < m.size()) m.erase(at, 1 + rng() % 16); break;
                default: m.insert(at, m.substr(rng() % m.size(), 1 + rng() % 40)); break;
            }
            spit(tmp, m);
            int rc = ff_read_set_file(tmp.c_str(), s, err);
            expect(rc == FF_OK || rc == FF_ERR_PARSE, "mutated file: parse or FF_ERR_PARSE");
            (rc == FF_OK ? parsed : refused)++;
        }
    }
    FfSetFile s;
    expect(ff_read_set_file((scratch + "/none.txt").c_str(), s, err) == FF_ERR_IO, "missing set is FF_ERR_IO");
    // Descriptors with out-of-range fields.
    const char* bad[] = {"0 n 64 64 16 32 2 2 1 4 1 8 1 0 3", "0 n 64 64 16 31 2 2 1 4 1 8 1 0 1",
                         "0 n 64 64 16 32 2147483647 2147483647 2147483647 4 1 8 1 0 1",
                         "0 n 64 64 16 32 2 2 1 3 1 8 1 0 1", "-1 n 64 64 16 32 2 2 1 4 1 8 1 0 1",
                         "0 n-x 64 64 16 32 2 2 1 4 1 8 1 0 1", "0 n 64 64 16 32 2 2 1 4 1 8 1 0"};
    for (const char* b : bad) {
        std::istringstream is(b);
        FfDesc d;
        expect(!ff_parse_descriptor(is, d), b);
    }
    printf("parser: %ld mutated files parsed, %ld refused\n", parsed, refused);
}

std::vector<double> random_table(std::mt19937_64& rng, int nv, int ns, double p_fail)
{
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<double> t((size_t)nv * ns);
    for (double& x : t) x = u(rng) < p_fail ? INFINITY : 0.01 + u(rng) * 10.0;
    return t;
}

// The tuning routines on random tables (failed entries included), with
// every output buffer sized exactly, plus argument errors.
void ptune_cases()
{
    std::mt19937_64 rng(15277);
    for (int trial = 0; trial < 400; ++trial) {
        const int nv = 1 + (int)(rng() % 14), ns = 1 + (int)(rng() % 9);
        const std::vector<double> t = random_table(rng, nv, ns, trial % 3 == 0 ? 0.2 : 0.0);
        std::vector<double> best(ns), worst(ns), slow((size_t)nv * ns), speed((size_t)nv * ns);
        std::vector<int> best_id(ns);
        expect(ptune_postprocess(nv, ns, t.data(), best.data(), worst.data(), best_id.data(), slow.data(),
                                 speed.data()) >= 0, "postprocess");
        const int k = 1 + (int)(rng() % (nv + 1));
        std::vector<int> shapes(ns);
        for (int s = 0; s < ns; ++s) shapes[s] = s;
        const int nsel = 1 + (int)(rng() % ns);
        for (int method = -1; method <= 1; ++method) {
            std::vector<int> kappa(k);
            double cost = 0;
            int64_t evals = 0;
            int got = ptune_select(nv, ns, t.data(), nsel, shapes.data(), k, method, kappa.data(), &cost, &evals);
            expect(got >= 0 && got <= k, "select size");
            if (got > 0) {
                double c2 = 0;
                expect(ptune_cost(nv, ns, t.data(), got, kappa.data(), nsel, shapes.data(), &c2) >= 0, "cost");
                std::vector<int> win(nsel);
                expect(ptune_assign(nv, ns, t.data(), got, kappa.data(), nsel, shapes.data(), win.data()) >= 0,
                       "assign");
            }
            std::vector<double> w(nsel, 1.0 + (double)(rng() % 5));
            double total = 0;
            got = ptune_select_total(nv, ns, t.data(), nsel, shapes.data(), w.data(), k, method, kappa.data(),
                                     &total, &evals);
            expect(got >= 0 && got <= k, "select_total size");
        }
        {
            const int kk = 1 + (int)(rng() % nsel);
            std::vector<int> init(kk), kappa(kk), assign(nsel);
            for (int c = 0; c < kk; ++c) init[c] = c;
            int iters = 0;
            int got = ptune_kmeans(nv, ns, t.data(), nsel, shapes.data(), kk, init.data(), 50, kappa.data(),
                                   assign.data(), &iters);
            expect(got >= 0 && got <= kk, "kmeans size");
        }
        {
            const int kk = 1 + (int)(rng() % nsel);
            std::vector<double> feat((size_t)nsel * 3);
            for (double& f : feat) f = (double)(rng() % 4);
            std::vector<int> kappa(kk), leaf(nsel), nfeat(2 * kk - 1), child(2 * (2 * kk - 1)), lvar(kk);
            std::vector<double> thr(2 * kk - 1);
            int got = ptune_tree(nv, ns, t.data(), nsel, shapes.data(), 3, feat.data(), kk, kappa.data(),
                                 leaf.data(), nfeat.data(), thr.data(), child.data(), lvar.data());
            expect(got >= 0 && got <= kk, "tree size");
            if (got > 0) {
                const double x[3] = {(double)(rng() % 5), 1.5, -1.0};
                // The tree holds 2 * leaves - 1 nodes; leaves may be fewer than kk.
                int leaves = 0;
                for (int n = 0; n < 2 * kk - 1; ++n)
                    if (nfeat[n] == -1) ++leaves;
                if (leaves > 0)
                    expect(ptune_tree_route(2 * leaves - 1, nfeat.data(), thr.data(), child.data(), 3, x) >= 0,
                           "tree route");
            }
        }
        {
            const int ntrain = 1 + (int)(rng() % 8), km = 1 + (int)(rng() % 5);
            std::vector<int64_t> mnk((size_t)ntrain * 3), gt((size_t)ntrain * km), gq(km);
            for (int64_t& x : mnk) x = 1 + (int64_t)(rng() % 5000);
            for (int64_t& x : gt) x = (int64_t)(rng() % 3000);
            for (int64_t& x : gq) x = (int64_t)(rng() % 3000);
            std::vector<int> members(km);
            for (int j = 0; j < km; ++j) members[j] = 3 * j + 1;
            std::vector<double> cost = random_table(rng, ntrain, km, 0.2);
            for (double& c : cost) c = std::isinf(c) ? c : std::log(1.0 + c);
            const int64_t M = (int64_t)(rng() % 9000), N = 1 + (int64_t)(rng() % 9000), K = (int64_t)(rng() % 9000);
            expect(ptune_nearest(ntrain, mnk.data(), M, N, K) >= 0, "nearest");
            const int id = ptune_dispatch(ntrain, mnk.data(), km, members.data(), cost.data(), gt.data(), gq.data(),
                                          256, M, N, K);
            expect(id >= 1, "dispatch returns a member");
            expect(ptune_dispatch(ntrain, mnk.data(), km, members.data(), cost.data(), nullptr, nullptr, 0, M, N, K)
                       >= 1, "dispatch without correction");
        }
    }
    // Argument errors must be reported, not dereferenced.
    expect(ptune_postprocess(-1, 3, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) < 0, "postprocess args");
    expect(ptune_select(3, 3, nullptr, 3, nullptr, 2, 0, nullptr, nullptr, nullptr) < 0, "select args");
    expect(ptune_cost(3, 3, nullptr, 1, nullptr, 0, nullptr, nullptr) < 0, "cost args");
    expect(ptune_nearest(0, nullptr, 1, 1, 1) < 0, "nearest args");
    expect(ptune_dispatch(0, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, 1, 1, 1) < 0, "dispatch args");
    expect(ptune_tree_route(0, nullptr, nullptr, nullptr, 3, nullptr) < 0, "tree route args");
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: %s <sets dir> <variants dir> <scratch dir>\n", argv[0]);
        return 2;
    }
    parser_cases(argv[1], argv[2], argv[3]);
    ptune_cases();
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
