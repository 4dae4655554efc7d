// Kernel-shape tuning table: the launch shapes picked by timing (the
// multi-right-hand-side GEMM's K split and stage depth, the symmetric
// mat-vec's tile edge), keyed by kernel, precision and a size class, shared
// by every context of the process and kept in a text file between
// processes, so that all problems and serving workers of one size class use
// the same shapes (and so the same summation order) once a class is tuned.
//
// File: $BEMTX_TUNE_FILE, else $XDG_CACHE_HOME/bemtx/tune-gfx950.txt, else
// $HOME/.cache/bemtx/tune-gfx950.txt; one "key value..." line per entry.  An
// unreadable or unwritable file only means the shapes are tuned again.
#include <cerrno>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <vector>

#include "internal.h"

namespace bemtx {

namespace {

struct Table {
    std::mutex mu;
    std::condition_variable cv;
    bool loaded = false;
    std::map<std::string, std::vector<int>> entries;
    std::set<std::string> busy;   // keys being tuned right now (other callers wait for them)
};

Table &table()
{
    static Table *t = new Table;   // never destroyed: callers may run during process exit
    return *t;
}

std::string tune_path()
{
    if (const char *f = std::getenv("BEMTX_TUNE_FILE")) return f;
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) dir = std::string(x) + "/bemtx";
    else if (const char *h = std::getenv("HOME")) dir = std::string(h) + "/.cache/bemtx";
    else return "";
    return dir + "/tune-gfx950.txt";
}

void load_locked(Table &t)
{
    if (t.loaded) return;
    t.loaded = true;
    const std::string path = tune_path();
    if (path.empty()) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        if (!(is >> key) || key.empty() || key[0] == '#') continue;
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        if (!v.empty()) t.entries[key] = v;
    }
}

void save_locked(const Table &t)
{
    const std::string path = tune_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {   // create the directory chain
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "# bemtx kernel shapes tuned on gfx950: key value...\n";
        for (const auto &e : t.entries) {
            f << e.first;
            for (int x : e.second) f << ' ' << x;
            f << '\n';
        }
        if (!f) return;
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

int tune_class(int64_t n)
{
    // quarter octaves: shapes tuned for n serve n within about 19 %
    return n <= 1 ? 0 : (int)std::lround(4.0 * std::log2((double)n));
}

bem_status tuned(const std::string &key, std::vector<int> &value, const std::function<bem_status(std::vector<int> &)> &tune,
                 const std::function<bool(const std::vector<int> &)> &valid)
{
    Table &t = table();
    {
        std::unique_lock<std::mutex> lk(t.mu);
        load_locked(t);
        for (;;) {
            auto it = t.entries.find(key);
            if (it != t.entries.end() && (!valid || valid(it->second))) {
                value = it->second;
                return BEM_OK;
            }
            if (!t.busy.count(key)) break;
            t.cv.wait(lk);   // another context is tuning this class: use its result
        }
        t.busy.insert(key);
    }
    std::vector<int> v;
    bem_status s = tune(v);
    std::lock_guard<std::mutex> lk(t.mu);
    t.busy.erase(key);
    if (s == BEM_OK && !v.empty()) {
        t.entries[key] = v;
        save_locked(t);
        value = v;
    }
    t.cv.notify_all();
    return s;
}

std::string tune_table_text()
{
    Table &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    load_locked(t);
    std::string out;
    for (const auto &e : t.entries) {
        out += e.first;
        for (int x : e.second) out += ' ' + std::to_string(x);
        out += '\n';
    }
    return out;
}

}  // namespace bemtx
