// The autotuner's choices as a JSON file, so that a later process starts
// tuned. Part of the libxeng.so translation unit (included by xeng.hip after
// the autotuner).
//
// Format (written by xeng_tuning_save, read by xeng_tuning_load):
//   {"format": "xeng-tuning", "version": 1,
//    "subarrays": [{"arch": "gfx950", "n_inputs": N, "n_chans": F, "n_time": T,
//                   "in_bits": B, "engine": E, "kernel": "small_n", "tile": 64}, ...],
//    "batches": [{"arch": "gfx950", "shapes": [[N, F, T, B, E], ...],
//                 "kernels": [["small_n", 64], ...],
//                 "workgroups_per_cu": 2, "order": 1}, ...]}
// A subarray entry is the choice for that shape alone; a batch entry the
// choices and schedule for that list of shapes together. Entries of another
// architecture are kept (and written back) but never applied.
//
// With the environment variable XENG_TUNING_FILE set, the first xeng_create
// of a process loads that file (if it exists; a file that cannot be read is
// ignored) and every xeng_autotune writes the whole cache back to it.
#pragma once

#include <stdlib.h>
#include <unistd.h>

namespace {

std::string device_arch(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// ---- a small JSON reader (objects, arrays, strings, numbers, literals)
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const char *key) const
    {
        for (const auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JReader {
    const char *p, *end;
    std::string err;
    bool fail_at(const char *what)
    {
        if (err.empty()) err = what;
        return false;
    }
    void ws()
    {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool lit(const char *w)
    {
        const size_t n = strlen(w);
        if ((size_t)(end - p) < n || strncmp(p, w, n) != 0) return fail_at("bad literal");
        p += n;
        return true;
    }
    bool string(std::string &out)
    {
        if (p >= end || *p != '"') return fail_at("expected a string");
        ++p;
        out.clear();
        while (p < end && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (p >= end) break;
                const char c = *p;
                out += c == 'n' ? '\n' : c == 't' ? '\t' : c; // \" \\ \/ and the rest verbatim
            } else {
                out += *p;
            }
            ++p;
        }
        if (p >= end) return fail_at("unterminated string");
        ++p;
        return true;
    }
    bool value(JVal &v, int depth)
    {
        if (depth > 16) return fail_at("nesting too deep");
        ws();
        if (p >= end) return fail_at("unexpected end");
        if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
                return true;
            }
            for (;;) {
                ws();
                std::string k;
                if (!string(k)) return false;
                ws();
                if (p >= end || *p != ':') return fail_at("expected ':'");
                ++p;
                v.obj.emplace_back(k, JVal());
                if (!value(v.obj.back().second, depth + 1)) return false;
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == '}') {
                    ++p;
                    return true;
                }
                return fail_at("expected ',' or '}'");
            }
        }
        if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
                return true;
            }
            for (;;) {
                v.arr.emplace_back();
                if (!value(v.arr.back(), depth + 1)) return false;
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == ']') {
                    ++p;
                    return true;
                }
                return fail_at("expected ',' or ']'");
            }
        }
        if (*p == '"') {
            v.kind = JVal::STR;
            return string(v.str);
        }
        if (*p == 't') {
            v.kind = JVal::BOOL;
            v.num = 1;
            return lit("true");
        }
        if (*p == 'f') {
            v.kind = JVal::BOOL;
            return lit("false");
        }
        if (*p == 'n') return lit("null");
        char *q = nullptr;
        std::string tok(p, (size_t)std::min<ptrdiff_t>(end - p, 40));
        v.num = strtod(tok.c_str(), &q);
        if (q == tok.c_str()) return fail_at("bad value");
        v.kind = JVal::NUM;
        p += q - tok.c_str();
        return true;
    }
};

bool j_int(const JVal *v, int &out)
{
    if (!v || v->kind != JVal::NUM || v->num != (double)(int)v->num) return false;
    out = (int)v->num;
    return true;
}

int fam_from_name(const std::string &n)
{
    for (int f : {FAM_REG, FAM_WG, FAM_W1, FAM_W2, FAM_SN})
        if (n == fam_name(f)) return f;
    return -1;
}

int tile_of(const SubChoice &c)
{
    return c.fam == FAM_REG ? 32 * c.wt : (c.fam == FAM_W2 || c.fam == FAM_SN ? 64 : 128);
}

bool choice_from(const std::string &kernel, int tile, SubChoice &c)
{
    c.fam = fam_from_name(kernel);
    if (c.fam < 0) return false;
    if (c.fam == FAM_REG) {
        if (tile != 32 && tile != 64 && tile != 128) return false;
        c.wt = tile / 32;
    } else {
        c.wt = 4;
    }
    return true;
}

bool shape_from(const JVal &a, SubKey &k)
{
    if (a.kind != JVal::ARR || a.arr.size() != 5) return false;
    int v[5];
    for (int q = 0; q < 5; ++q)
        if (!j_int(&a.arr[q], v[q])) return false;
    k = SubKey{v[0], v[1], v[2], v[3], v[4]};
    return true;
}

std::string json_str(const std::string &s)
{
    std::string o = "\"";
    for (char c : s) {
        if (c == '"' || c == '\\') o += '\\';
        if ((unsigned char)c >= 0x20) o += c;
    }
    return o + "\"";
}

// Parse a tuning file into the cache; the caller holds g_tune_mu.
int tuning_parse(const std::string &text, const char *path, int &n_loaded)
{
    JReader r{text.data(), text.data() + text.size(), {}};
    JVal root;
    if (!r.value(root, 0)) return fail(XENG_EINVAL, "%s: not JSON (%s)", path, r.err.c_str());
    const JVal *fmt = root.get("format");
    int version = 0;
    if (root.kind != JVal::OBJ || !fmt || fmt->kind != JVal::STR || fmt->str != "xeng-tuning" ||
        !j_int(root.get("version"), version) || version != 1)
        return fail(XENG_EINVAL, "%s: not an xeng-tuning version 1 file", path);
    std::map<ArchKey, SubChoice> subs;
    std::map<ArchSet, std::vector<SubChoice>> sets;
    std::map<ArchSet, SchedChoice> scheds;
    if (const JVal *a = root.get("subarrays")) {
        if (a->kind != JVal::ARR) return fail(XENG_EINVAL, "%s: \"subarrays\" is not a list", path);
        for (size_t q = 0; q < a->arr.size(); ++q) {
            const JVal &e = a->arr[q];
            const JVal *arch = e.get("arch"), *kern = e.get("kernel");
            int v[5], tile = 0;
            SubChoice c;
            if (!arch || arch->kind != JVal::STR || !kern || kern->kind != JVal::STR ||
                !j_int(e.get("n_inputs"), v[0]) || !j_int(e.get("n_chans"), v[1]) ||
                !j_int(e.get("n_time"), v[2]) || !j_int(e.get("in_bits"), v[3]) ||
                !j_int(e.get("engine"), v[4]) || !j_int(e.get("tile"), tile) ||
                !choice_from(kern->str, tile, c))
                return fail(XENG_EINVAL, "%s: subarray entry %zu is malformed", path, q);
            subs[ArchKey{arch->str, SubKey{v[0], v[1], v[2], v[3], v[4]}}] = c;
        }
    }
    if (const JVal *a = root.get("batches")) {
        if (a->kind != JVal::ARR) return fail(XENG_EINVAL, "%s: \"batches\" is not a list", path);
        for (size_t q = 0; q < a->arr.size(); ++q) {
            const JVal &e = a->arr[q];
            const JVal *arch = e.get("arch"), *sh = e.get("shapes"), *ks = e.get("kernels");
            int wg = 0, order = 0;
            bool ok = arch && arch->kind == JVal::STR && sh && sh->kind == JVal::ARR && ks &&
                      ks->kind == JVal::ARR && sh->arr.size() == ks->arr.size() && !sh->arr.empty() &&
                      sh->arr.size() <= (size_t)MAX_SUBS && j_int(e.get("workgroups_per_cu"), wg) &&
                      j_int(e.get("order"), order) && wg >= 1 && wg <= 8 && (order == 0 || order == 1);
            std::vector<SubKey> keys;
            std::vector<SubChoice> cs;
            for (size_t k = 0; ok && k < sh->arr.size(); ++k) {
                SubKey key;
                SubChoice c;
                const JVal &kc = ks->arr[k];
                int tile = 0;
                ok = shape_from(sh->arr[k], key) && kc.kind == JVal::ARR && kc.arr.size() == 2 &&
                     kc.arr[0].kind == JVal::STR && j_int(&kc.arr[1], tile) &&
                     choice_from(kc.arr[0].str, tile, c);
                keys.push_back(key);
                cs.push_back(c);
            }
            if (!ok) return fail(XENG_EINVAL, "%s: batch entry %zu is malformed", path, q);
            sets[ArchSet{arch->str, keys}] = cs;
            scheds[ArchSet{arch->str, keys}] = SchedChoice{wg, order};
        }
    }
    // nothing is merged unless the whole file parsed
    for (auto &kv : subs) g_tune_sub[kv.first] = kv.second;
    for (auto &kv : sets) g_tune_set[kv.first] = kv.second;
    for (auto &kv : scheds) g_tune_sched[kv.first] = kv.second;
    n_loaded = (int)(subs.size() + sets.size());
    return XENG_OK;
}

// The whole cache as a tuning file; the caller holds g_tune_mu.
std::string tuning_text(int &n_entries)
{
    std::string js = "{\"format\": \"xeng-tuning\", \"version\": 1,\n \"subarrays\": [";
    char buf[512];
    n_entries = 0;
    bool first = true;
    for (const auto &kv : g_tune_sub) {
        const SubKey &k = kv.first.second;
        snprintf(buf, sizeof buf,
                 "%s\n  {\"arch\": %s, \"n_inputs\": %d, \"n_chans\": %d, \"n_time\": %d, "
                 "\"in_bits\": %d, \"engine\": %d, \"kernel\": \"%s\", \"tile\": %d}",
                 first ? "" : ",", json_str(kv.first.first).c_str(), k.n, k.f, k.t, k.b, k.e,
                 fam_name(kv.second.fam), tile_of(kv.second));
        js += buf;
        first = false;
        ++n_entries;
    }
    js += "],\n \"batches\": [";
    first = true;
    for (const auto &kv : g_tune_set) {
        auto sc = g_tune_sched.find(kv.first);
        const SchedChoice sch = sc != g_tune_sched.end() ? sc->second : SchedChoice{WG_PER_CU, 0};
        js += first ? "\n  {\"arch\": " : ",\n  {\"arch\": ";
        js += json_str(kv.first.first) + ", \"shapes\": [";
        for (size_t q = 0; q < kv.first.second.size(); ++q) {
            const SubKey &k = kv.first.second[q];
            snprintf(buf, sizeof buf, "%s[%d, %d, %d, %d, %d]", q ? ", " : "", k.n, k.f, k.t, k.b, k.e);
            js += buf;
        }
        js += "], \"kernels\": [";
        for (size_t q = 0; q < kv.second.size(); ++q) {
            snprintf(buf, sizeof buf, "%s[\"%s\", %d]", q ? ", " : "", fam_name(kv.second[q].fam),
                     tile_of(kv.second[q]));
            js += buf;
        }
        snprintf(buf, sizeof buf, "], \"workgroups_per_cu\": %d, \"order\": %d}", sch.wg_per_cu, sch.order);
        js += buf;
        first = false;
        ++n_entries;
    }
    js += "]}\n";
    return js;
}

int tuning_write(const char *path, int &n_entries)
{
    std::string text;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        text = tuning_text(n_entries);
    }
    // write a sibling file, then rename it over the target
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *fp = fopen(tmp.c_str(), "wb");
    if (!fp) return fail(XENG_EINVAL, "cannot write %s", tmp.c_str());
    const bool ok = fwrite(text.data(), 1, text.size(), fp) == text.size();
    if (fclose(fp) != 0 || !ok) {
        remove(tmp.c_str());
        return fail(XENG_EINVAL, "cannot write %s", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(XENG_EINVAL, "cannot rename %s to %s", tmp.c_str(), path);
    }
    return XENG_OK;
}

int tuning_read(const char *path, int &n_loaded)
{
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(XENG_EINVAL, "cannot open %s", path);
    std::string text;
    char buf[65536];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, fp)) > 0) {
        text.append(buf, n);
        if (text.size() > ((size_t)64 << 20)) {
            fclose(fp);
            return fail(XENG_EINVAL, "%s: larger than 64 MiB", path);
        }
    }
    fclose(fp);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return tuning_parse(text, path, n_loaded);
}

std::once_flag g_tuning_autoload;

void tuning_file_autoload()
{
    std::call_once(g_tuning_autoload, []() {
        const char *path = getenv("XENG_TUNING_FILE");
        if (!path || !*path) return;
        FILE *fp = fopen(path, "rb");
        if (!fp) return; // nothing tuned yet
        fclose(fp);
        int n = 0;
        (void)tuning_read(path, n); // an unreadable file is ignored
    });
}

void tuning_file_autosave()
{
    const char *path = getenv("XENG_TUNING_FILE");
    if (!path || !*path) return;
    int n = 0;
    (void)tuning_write(path, n);
}

} // namespace

extern "C" {

int xeng_tuning_load(const char *path, int *n_entries)
{
    if (!path) return fail(XENG_EINVAL, "path is NULL");
    int n = 0;
    const int rc = tuning_read(path, n);
    if (n_entries) *n_entries = rc ? 0 : n;
    return rc;
}

int xeng_tuning_save(const char *path, int *n_entries)
{
    if (!path) return fail(XENG_EINVAL, "path is NULL");
    int n = 0;
    const int rc = tuning_write(path, n);
    if (n_entries) *n_entries = rc ? 0 : n;
    return rc;
}

int xeng_tuning_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_sub.clear();
    g_tune_set.clear();
    g_tune_sched.clear();
    return XENG_OK;
}

} // extern "C"
