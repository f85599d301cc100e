// Parsing of variant descriptors, manifests and variant-set files (host
// only; declared in setfile.h).

#include "setfile.h"

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "../../include/fewfit.h"

namespace {

int parse_fail(std::string& err, int code, const char* fmt, const char* a = "", long b = 0, const char* c = "")
{
    char buf[512];
    snprintf(buf, sizeof buf, fmt, a, b, c);
    err = buf;
    return code;
}

}  // namespace

bool ff_parse_descriptor(std::istream& is, FfDesc& v)
{
    if (!(is >> v.id >> v.name >> v.mwg >> v.nwg >> v.kwg >> v.mi >> v.wm >> v.wn >> v.sk >> v.vw >> v.lds >> v.gm >>
          v.sg >> v.prec >> v.pd))
        return false;
    if (v.pd < 1 || v.pd > 2) return false;
    if (v.id < 0 || v.mwg <= 0 || v.nwg <= 0 || v.kwg <= 0 || (v.mi != 16 && v.mi != 32) || v.wm <= 0 ||
        v.wn <= 0 || v.sk <= 0 || (v.vw != 1 && v.vw != 2 && v.vw != 4) || v.lds < 0 || v.lds > 2 ||
        (v.lds == 2 && v.vw != 4) || v.gm <= 0 || v.sg < 1 || v.sg > 64 || v.prec < 0 || v.prec > 4)
        return false;
    // Each factor of the thread count is positive here; bound them before
    // multiplying so that the product cannot overflow.
    if (v.wm > 1024 || v.wn > 1024 || v.sk > 1024 || (int64_t)v.wm * v.wn * v.sk > 16) return false;
    if (v.mwg > 4096 || v.nwg > 4096 || v.kwg > 4096) return false;
    if (v.prec > 0 && (v.sk != 1 || v.lds < 1)) return false;
    if (v.name.empty()) return false;
    for (char c : v.name)
        if (!(isalnum((unsigned char)c) || c == '_')) return false;
    return true;
}

int ff_read_manifest(const char* dir, std::vector<FfDesc>& out, std::string& err)
{
    out.clear();
    const std::string path = std::string(dir) + "/manifest.txt";
    std::ifstream f(path);
    if (!f) return parse_fail(err, FF_ERR_IO, "cannot open %s", path.c_str());
    std::string line;
    long lineno = 0;
    while (std::getline(f, line)) {
        ++lineno;
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        FfDesc v;
        if (!ff_parse_descriptor(is, v)) return parse_fail(err, FF_ERR_PARSE, "%smanifest line %ld: bad descriptor", "", lineno);
        out.push_back(v);
    }
    return FF_OK;
}

// Set file format (text, '#' comments):
//   fewfit-set 1
//   arch <gfx name>
//   codedir <dir>          code objects, relative to the set file's directory
//   form <name>            optional: fp32 (default), bf16x3, bf16x6, fp16s or fp16x3,
//                          and every member is of that form; or mixed, members of
//                          any form (a set chosen for an accuracy target)
//   variant <descriptor>   k lines, descriptor as in the manifest
//   rule <M> <N> <K> <id> <c_1> ... <c_k>
//                          one line per training shape (after the variant
//                          lines): its winner, a member, and every member's
//                          log-slowdown on it ("inf" where it failed)
//   end
int ff_read_set_file(const char* path, FfSetFile& set, std::string& err)
{
    set = FfSetFile{};
    std::ifstream f(path);
    if (!f) return parse_fail(err, FF_ERR_IO, "cannot open set file %s", path);
    std::vector<int> ids;
    std::string line;
    bool header = false, ended = false;
    long lineno = 0;
    while (std::getline(f, line)) {
        ++lineno;
        size_t h = line.find('#');
        if (h != std::string::npos) line = line.substr(0, h);
        std::istringstream is(line);
        std::string key;
        if (!(is >> key)) continue;
        if (ended) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: text after 'end'", path, lineno);
        if (!header) {
            int ver = 0;
            if (key != "fewfit-set" || !(is >> ver) || ver != 1)
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: expected 'fewfit-set 1'", path, lineno);
            header = true;
            continue;
        }
        std::string extra;
        if (key == "arch") {
            if (!(is >> set.arch)) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: arch needs a value", path, lineno);
        } else if (key == "codedir") {
            if (!(is >> set.codedir)) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: codedir needs a value", path, lineno);
        } else if (key == "form") {
            std::string name;
            static const char* names[kFfForms] = {"fp32", "bf16x3", "bf16x6", "fp16s", "fp16x3", "mixed"};
            if (!(is >> name)) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: form needs a value", path, lineno);
            set.form = -1;
            for (int i = 0; i < kFfForms; ++i)
                if (name == names[i]) set.form = i;
            if (set.form < 0) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: unknown form '%s'", path, lineno, name.c_str());
        } else if (key == "variant") {
            FfDesc v;
            if (!ff_parse_descriptor(is, v)) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: bad variant descriptor", path, lineno);
            if (std::find(ids.begin(), ids.end(), v.id) != ids.end())
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: duplicate variant", path, lineno);
            if (!set.shapes.empty())
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: variant lines must precede the rules", path, lineno);
            if (set.members.size() >= (size_t)kFfMaxMembers)
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: more than 64 members", path, lineno);
            set.members.push_back(v);
            ids.push_back(v.id);
        } else if (key == "rule") {
            long long m, n, k;
            int id;
            if (!(is >> m >> n >> k >> id) || m < 1 || n < 1 || k < 1 || m > INT32_MAX || n > INT32_MAX ||
                k > INT32_MAX)
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: bad rule", path, lineno);
            const auto pos = std::find(ids.begin(), ids.end(), id);
            if (pos == ids.end())
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: rule names a variant outside the set", path, lineno);
            std::vector<double> c(ids.size());
            for (size_t j = 0; j < c.size(); ++j) {
                std::string tok;
                if (!(is >> tok)) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: rule needs a cost per member", path, lineno);
                char* end = nullptr;
                c[j] = (tok == "inf") ? INFINITY : std::strtod(tok.c_str(), &end);
                if (tok != "inf" && (end == tok.c_str() || *end != '\0' || !(c[j] >= 0.0) || !std::isfinite(c[j])))
                    return parse_fail(err, FF_ERR_PARSE, "%s:%ld: bad member cost '%s'", path, lineno, tok.c_str());
            }
            if (c[pos - ids.begin()] != *std::min_element(c.begin(), c.end()))
                return parse_fail(err, FF_ERR_PARSE, "%s:%ld: rule winner is not the cheapest member", path, lineno);
            set.shapes.push_back({m, n, k});
            set.winners.push_back(id);
            set.cost.insert(set.cost.end(), c.begin(), c.end());
        } else if (key == "end") {
            ended = true;
        } else {
            return parse_fail(err, FF_ERR_PARSE, "%s:%ld: unknown key '%s'", path, lineno, key.c_str());
        }
        if (key != "end" && (is >> extra)) return parse_fail(err, FF_ERR_PARSE, "%s:%ld: trailing text", path, lineno);
    }
    if (!header) return parse_fail(err, FF_ERR_PARSE, "%s: empty set file", path);
    if (!ended) return parse_fail(err, FF_ERR_PARSE, "%s: missing 'end' (truncated file?)", path);
    if (set.arch.empty() || set.codedir.empty() || set.members.empty() || set.shapes.empty())
        return parse_fail(err, FF_ERR_PARSE, "%s: needs arch, codedir, at least one variant and one rule", path);
    for (const FfDesc& v : set.members)
        if (set.form != kFfPrecForms && v.prec != set.form)
            return parse_fail(err, FF_ERR_PARSE, "%s: a variant is not of the set's form", path);
    return FF_OK;
}
